/*
 * lst.h -- C ABI of the MI355X (gfx950) Line Segment Tracking library.
 *
 * Line Segment Tracking (arXiv:2207.08207) builds track candidates bottom-up
 * (Section 2.1): mini-doublets (MD, hit pairs of one pT module, Section 2.2),
 * line segments (LS, two MDs in modules linked by the module map, Section
 * 2.2), triplets and quintuplets (T3/T5, segments and triplets sharing an MD,
 * Section 2.3), pixel line segments and pixel triplets/quintuplets (pLS,
 * pT3/pT5, Section 2.4), then removes duplicates and cross-cleans them into
 * track candidates in the order pT5, pT3, T5, pLS (Section 2.5).  Hits and
 * the module map go in; lists of hit indices come out (Section 4.2, whose
 * flowchart starts from hits in GPU memory and ends by copying the track
 * candidates to the host).
 *
 * Conventions
 *  - Every function returns lst_status: LST_OK (0) or a negative error.  On
 *    error lst_last_error() returns a message (thread-local, valid until the
 *    next call on the same thread).  No C++ exception crosses this boundary.
 *  - Geometry inputs are HOST pointers, copied during lst_load_geometry.
 *  - Event inputs are DEVICE pointers (already in HBM), read while the chain
 *    runs on the caller's stream; they must stay valid until the event has
 *    completed (lst_build_event returns after completion).
 *  - Device memory for one event comes from a caller-owned workspace (for
 *    example a torch uint8 tensor) of at least lst_workspace_bytes() bytes;
 *    the library never allocates device memory per event.  The workspace
 *    holds the event's objects and must outlive the lst_event that uses it.
 *  - Hit indices in every output are 0-based positions in the caller's hit
 *    arrays.  Stage ids: 0 MD, 1 LS, 2 T3, 3 T5, 4 pLS, 5 pT3, 6 pT5, 7 TC.
 *  - One geometry may serve many events and threads; one lst_event must not
 *    be used by two threads at once.
 */
#ifndef LST_H
#define LST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LST_OK = 0,
  LST_E_INVALID = -1,   /* bad argument or invalid input data (e.g. module id out of range, NaN) */
  LST_E_NOMEM = -2,     /* workspace too small, or a host/device allocation at setup failed */
  LST_E_CAPACITY = -3,  /* an object count exceeded its capacity; required counts are reported */
  LST_E_DEVICE = -4,    /* a HIP runtime call failed */
  LST_E_STATE = -5      /* call made in the wrong state (e.g. event not complete) */
} lst_status;

typedef struct lst_geometry_s *lst_geometry; /* opaque, library-owned, device-resident */
typedef struct lst_event_s *lst_event;       /* opaque, library-owned host handle */
typedef struct lst_plan_s *lst_plan;         /* opaque: a captured batch chain (HIP graph) */
typedef struct lst_server_s *lst_server;     /* opaque: a serving loop */

/* Detector description (Section 1: bi-layer pT modules) and module map
 * (Section 2.2).  All arrays are HOST memory, length n_modules unless noted.
 *  subdet   0 barrel, 1 endcap
 *  layer    barrel layer 1..6 or endcap disk 1..5
 *  side     0 barrel, -1 / +1 endcap side
 *  type     0 PS (macro-pixel), 1 2S (strip)
 *  pos_lo   barrel: radius of the lower sensor [cm]; endcap: |z| of the lower sensor plane
 *  pos_up   the same for the upper sensor
 *  lmin,lmax  range of the long coordinate: z in the barrel, r in the endcap [cm]
 *  map_offsets  n_modules + 1 CSR offsets; map_targets  n_edges module ids,
 *               the modules of the next surface linked to each module (at
 *               most 128 per module; LST_E_INVALID otherwise). */
typedef struct {
  int32_t n_modules;
  const int32_t *subdet, *layer, *side, *type;
  const float *pos_lo, *pos_up, *lmin, *lmax;
  int32_t n_edges;
  const int32_t *map_offsets, *map_targets;
} lst_geometry_desc;

/* One event, all arrays in DEVICE memory (n_hits and n_seeds at most
 * 8,000,000 each; LST_E_INVALID beyond).
 *  x,y,z [n_hits] hit positions [cm]; module [n_hits] module id or -1 for a
 *  pixel hit; sensor [n_hits] 0 lower / 1 upper (ignored for pixel hits).
 *  Seeds (Section 2.4 pixel tracks; n_seeds may be 0 and the pointers NULL):
 *  px,py,pz [n_seeds] momentum at the innermost pixel hit [GeV]; q [n_seeds]
 *  charge +1/-1; hits4 [n_seeds x 4] pixel-hit indices, innermost first. */
typedef struct {
  int32_t n_hits;
  const float *x, *y, *z;
  const int32_t *module, *sensor;
  int32_t n_seeds;
  const float *px, *py, *pz;
  const int32_t *q, *hits4;
} lst_event_desc;

/* Object capacities of one event.  Counts beyond a capacity are never
 * truncated silently: the build returns LST_E_CAPACITY and
 * lst_get_stage_counts() reports the required counts. */
typedef struct {
  int64_t md, ls, t3, t5, pt3, pt5;
} lst_capacity;

/* Uploads the detector and module map and computes the per-module
 * mini-doublet windows on the device.  *out is owned by the caller and freed
 * with lst_release_geometry.  Errors: LST_E_INVALID (NULL pointer, negative
 * size, module id or CSR out of range), LST_E_DEVICE, LST_E_NOMEM. */
lst_status lst_load_geometry(const lst_geometry_desc *desc, lst_geometry *out);
lst_status lst_release_geometry(lst_geometry geom);

/* Default capacities for an event of n_hits hits and n_seeds seeds. */
lst_status lst_default_capacity(int32_t n_hits, int32_t n_seeds, lst_capacity *out);

/* Workspace size in bytes for an event of n_hits hits and n_seeds seeds
 * with the given capacities (NULL = defaults). */
lst_status lst_workspace_bytes(lst_geometry geom, int32_t n_hits, int32_t n_seeds, const lst_capacity *cap,
                               size_t *bytes);

/* Runs the whole chain for one event on `stream` (a hipStream_t; NULL = the
 * null stream) inside the caller's workspace and waits for it.  *out is a new
 * event handle (freed with lst_release_event) even when the status is
 * LST_E_CAPACITY or LST_E_INVALID (so the caller can read the counts).
 * Errors: LST_E_INVALID (arguments, or invalid hit/seed data detected on the
 * device), LST_E_NOMEM (ws_bytes too small), LST_E_CAPACITY, LST_E_DEVICE. */
lst_status lst_build_event(lst_geometry geom, const lst_event_desc *ev, const lst_capacity *cap, void *workspace,
                           size_t ws_bytes, void *stream, lst_event *out);

/* Allocation-free form of lst_build_event, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The event runs in the library's static workspace: one device
 * array of lst_static_workspace_bytes() bytes (256 MiB) per GPU, held from the
 * first call on that GPU until the process ends.  The call validates the
 * arguments and the event's workspace size on the host (LST_E_NOMEM, with the
 * bytes needed, when the event with its capacities does not fit; default
 * capacities fit events of up to about 200,000 hits), enqueues the chain on
 * `stream` and returns without waiting; it calls no hipMalloc, hipFree or
 * other allocating routine.  Outputs are caller DEVICE buffers: counts[0..2]
 * = number of track candidates, their total hit count, the chain's status
 * flags (0 = built; 1 invalid hit data, 2 invalid seed data, 4 capacity
 * exceeded); type[max_tc], offsets[max_tc + 1] and hits[max_tc_hits] are
 * written (as lst_get_track_candidates lays them out) only when the status
 * is 0 and both counts fit, so a caller reads counts after synchronizing the
 * stream and retries with larger buffers if needed.  Every call on one GPU
 * shares that GPU's workspace: calls that overlap on one GPU (different
 * streams or threads, or a call before the previous one's outputs were
 * consumed) race.  Errors: LST_E_INVALID (arguments, as lst_build_event),
 * LST_E_NOMEM (too large), LST_E_DEVICE (a HIP call failed). */
lst_status lst_build_event_static(lst_geometry geom, const lst_event_desc *ev, const lst_capacity *cap,
                                  void *stream, int32_t max_tc, int32_t max_tc_hits, int32_t *type,
                                  int32_t *offsets, int32_t *hits, int32_t *counts);
lst_status lst_static_workspace_bytes(size_t *bytes);

/* Asynchronous form: enqueues the chain on `stream` and returns at once.
 * Inputs and workspace must stay valid until lst_event_wait returns (or
 * lst_event_query reports completion).  The status of the build is returned
 * by lst_event_wait. */
lst_status lst_enqueue_event(lst_geometry geom, const lst_event_desc *ev, const lst_capacity *cap, void *workspace,
                             size_t ws_bytes, void *stream, lst_event *out);
/* 1 if the event's device work has completed, 0 if not (into *done). */
lst_status lst_event_query(lst_event ev, int32_t *done);
/* Blocks until the event's device work has completed; returns its status. */
lst_status lst_event_wait(lst_event ev);

/* Batched form: B independent events run by one launch sequence (each kernel
 * of the chain is launched once for the whole batch, events along the grid's
 * y dimension), inside one workspace of lst_batch_workspace_bytes() bytes
 * (n_hits / n_seeds: B entries; cap: B entries or NULL for defaults).  `out`
 * receives B event handles (each released with lst_release_event; waiting on
 * any of them waits for the batch).  Per event the results are identical to
 * lst_build_event's.  Section 4.2.2 fills the GPU with several events through
 * streams; here events also share each launch.  Errors as lst_build_event. */
lst_status lst_batch_workspace_bytes(lst_geometry geom, int32_t B, const int32_t *n_hits, const int32_t *n_seeds,
                                     const lst_capacity *cap, size_t *bytes);
lst_status lst_enqueue_batch(lst_geometry geom, int32_t B, const lst_event_desc *evs, const lst_capacity *cap,
                             void *workspace, size_t ws_bytes, void *stream, lst_event *out);

/* Captured plan: the batched chain for B slots, each sized for max_hits hits,
 * max_seeds seeds and capacities `cap` (NULL = defaults for those sizes), is
 * captured once into a HIP graph bound to `workspace`
 * (lst_plan_workspace_bytes() bytes; the caller keeps it alive until
 * lst_plan_release).  lst_plan_run(plan, n, evs, stream, out) writes the n
 * (<= B) event descriptors into the workspace header, replays the graph on
 * `stream` (NULL = the stream given at creation) and returns n event handles
 * (as lst_enqueue_batch; unused slots run as empty events).  A plan runs one
 * batch at a time: lst_plan_run returns LST_E_STATE while any event of the
 * previous run is still held.  Errors: LST_E_INVALID (an event larger than
 * the slots), LST_E_DEVICE (capture or launch failure), LST_E_NOMEM. */
lst_status lst_plan_workspace_bytes(lst_geometry geom, int32_t B, int32_t max_hits, int32_t max_seeds,
                                    const lst_capacity *cap, size_t *bytes);
lst_status lst_plan_create(lst_geometry geom, int32_t B, int32_t max_hits, int32_t max_seeds, const lst_capacity *cap,
                           void *workspace, size_t ws_bytes, void *stream, lst_plan *out);
lst_status lst_plan_run(lst_plan plan, int32_t n_events, const lst_event_desc *evs, void *stream, lst_event *out);
lst_status lst_plan_release(lst_plan plan);

/* Serving form: a request loop inside the library (its own host thread and
 * n_streams non-blocking HIP streams of default priority).  Requests arrive
 * with a time on the server clock (seconds since lst_server_create; a time
 * already past means "now"); arrived requests are admitted first come first
 * served, up to max_batch per launch sequence, whenever a stream is free and
 * the caller's device `pool` (pool_bytes, 256-byte aligned, kept alive until
 * lst_server_destroy) has room for the batch's footprint.  Batches on
 * different streams overlap on the device; an event's objects stay resident
 * in the pool until its handle is released, which returns the memory.
 * Per event the results are identical to lst_build_event's.  A request whose
 * objects overflow their capacities is run again, ahead of the queue, with
 * every capacity grown to 1.5 x the counts the overflowing run required (at
 * most three reruns; its arrival time and so its latency are kept); it is
 * reported LST_E_CAPACITY only after that, or LST_E_NOMEM when the grown
 * event no longer fits the pool.  When idle the server thread sleeps until a
 * submission, a released result or the next arrival.  Section 4.2.2's
 * multi-streaming is the paper's counterpart. */
typedef struct {
  int32_t n_streams; /* batches in flight, 1..64 (1 with max_batch 1 = the plain FIFO path) */
  int32_t max_batch; /* events per launch sequence, 1..1024 */
} lst_server_config;
typedef struct {
  int64_t id;        /* the caller's request id */
  lst_event event;   /* completed event (release with lst_release_event); NULL if it could not run */
  double arrival_s;  /* server-clock times: arrival, admission (batch enqueued), completion observed */
  double admit_s;
  double done_s;
  int32_t status;    /* LST_OK, LST_E_CAPACITY, LST_E_INVALID, LST_E_DEVICE, LST_E_NOMEM */
} lst_server_result;
lst_status lst_server_create(lst_geometry geom, const lst_server_config *cfg, void *pool, size_t pool_bytes,
                             lst_server *out);
/* Seconds since the server was created, on its clock. */
lst_status lst_server_now(lst_server srv, double *t);
/* Queues one event (device pointers valid until its result is released).
 * Errors: LST_E_INVALID (descriptor), LST_E_NOMEM (larger than the pool). */
lst_status lst_server_submit(lst_server srv, const lst_event_desc *ev, int64_t id, double arrival_s);
/* The same with the first attempt's capacities given (NULL: lst_default_capacity). */
lst_status lst_server_submit_with_capacity(lst_server srv, const lst_event_desc *ev, const lst_capacity *cap,
                                           int64_t id, double arrival_s);
/* Requests run again after a capacity overflow since the server was created. */
lst_status lst_server_reruns(lst_server srv, int64_t *n);
/* Moves up to `max` completed results to `out` (*n of them). */
lst_status lst_server_poll(lst_server srv, lst_server_result *out, int32_t max, int32_t *n);
/* Requests not yet admitted, and completed results not yet polled. */
lst_status lst_server_pending(lst_server srv, int32_t *queued, int32_t *ready);
/* Waits for the batches in flight, releases unpolled results, stops the loop.
 * Events still held by the caller stay readable but must be released before
 * the pool is freed. */
lst_status lst_server_destroy(lst_server srv);

/* Track candidates (Section 2.5) of a completed event, copied to HOST
 * buffers.  Two-call protocol: pass NULL arrays to get *n_tc and
 * *n_hits_total, then arrays of n_tc (type), n_tc + 1 (offsets) and
 * n_hits_total (hits).  type: 0 pT5, 1 pT3, 2 T5, 3 pLS, ordered by type,
 * then by seed index (pT5, pT3, pLS) or by the MDs' (module, lower hit,
 * upper hit) sequence (T5).  Hit lists: the four pixel hits innermost first,
 * then the lower and upper hit of each MD from inner to outer (14 / 10 / 10 / 4
 * hits).  Errors: LST_E_STATE if the event failed or is not complete. */
lst_status lst_get_track_candidates(lst_event ev, int32_t *n_tc, int32_t *n_hits_total, int32_t *type,
                                    int32_t *offsets, int32_t *hits);

/* Storage precision of the MD stubs (the tangential displacement and the
 * sensor separation of each mini-doublet, which the segment selection checks
 * against the chord's direction): 32 (float, the default) or 16 (IEEE
 * binary16, rounded to nearest even, read back as float) -- the
 * half-precision types Section 5 names as future work, for the quantity
 * whose precision the selection needs least.  Applies to chains enqueued
 * afterwards (plans created afterwards).  Errors: LST_E_INVALID for a NULL
 * geometry or bits other than 16 / 32. */
lst_status lst_set_stub_precision(lst_geometry geom, int32_t bits);

/* Transverse impact-parameter bound d0_max [cm] that every selection allows
 * for (MD windows, segment azimuth window and stub directions, the
 * azimuth-z pointing of triplets, quintuplets and extensions).  0.1 cm from
 * lst_load_geometry; Section 3 runs the same chain on displaced muons, for
 * which the bound is widened to their largest displacement.  Recomputes the
 * per-module MD windows on the device (synchronous) and applies to chains
 * enqueued afterwards (plans created afterwards); call it while no chain of
 * this geometry is in flight.  Errors: LST_E_INVALID for
 * a NULL geometry or a bound outside (0, 10]; LST_E_DEVICE. */
lst_status lst_set_impact_bound(lst_geometry geom, double d0_max);

/* Quintuplet chi2 cuts per category (Section 2.3 sets them empirically for
 * each category of quintuplets).  Category index c in [0, 1024) = sum over
 * the five anchor modules, innermost first, of kind_i * 4^i with kind
 * 0 barrel PS, 1 barrel 2S, 2 endcap PS, 3 endcap 2S.  xy[c] bounds the
 * five-anchor circle-fit chi2, rz[c] the r-z line chi2 (a quintuplet passes
 * when chi2 <= cut).  lst_load_geometry installs the library's calibrated
 * table; lst_set_t5_cuts replaces it with HOST arrays of 1024 floats (either
 * may be NULL: that half keeps the calibrated values) and applies to every
 * chain that starts afterwards, plans included; call it while no chain of
 * this geometry is in flight.  lst_get_t5_cuts copies the table in force to
 * two HOST arrays of 1024 floats; lst_get_default_t5_cuts copies the
 * calibrated table itself (host only: no geometry, no device needed).
 * Errors: LST_E_INVALID for a NULL geometry or output, or a NaN cut;
 * LST_E_DEVICE. */
lst_status lst_set_t5_cuts(lst_geometry geom, const float *xy, const float *rz);
lst_status lst_get_t5_cuts(lst_geometry geom, float *xy, float *rz);
lst_status lst_get_default_t5_cuts(float *xy, float *rz);

/* Track extensions (Section 2.5, last part): the final collection in which
 * a candidate with outer-tracker MDs (pT5, pT3, T5) is lengthened outward by
 * one triplet that shares its last two MDs (one MD added) or its last MD
 * (two added).  The paper gives no selection; this library takes the
 * triplet whose curvature agrees with the candidate's (seed resolution x3
 * for pT5 / pT3, the outer triplet's for a T5), whose anchors keep the
 * azimuth linear in z over the chain, and whose chain of all anchors passes
 * the quintuplet's x-y circle and (arc length, z) line fits widened to its
 * 4..7 anchors (chi2 <= 10 and 20/3 per degree of freedom); of those, the
 * one adding more MDs, then the smaller chi2 sum, then the smaller hit tuple
 * of the added MDs.
 *
 * lst_set_track_extensions(geom, 1) makes every chain enqueued afterwards on
 * `geom` (events, batches, servers; plans created afterwards) end with the
 * extension step; 0 (the default) leaves it out.  Errors: LST_E_INVALID for
 * a NULL geometry or a value other than 0 / 1. */
lst_status lst_set_track_extensions(lst_geometry geom, int32_t enable);

/* The extended collection of a completed event, copied to HOST buffers, in
 * the order and with the types of lst_get_track_candidates (two-call
 * protocol: NULL arrays to get *n_tc and *n_hits_total).  hits: each
 * candidate's hits as lst_get_track_candidates gives them, then the lower
 * and upper hit of each added MD, inner to outer; offsets [n_tc + 1];
 * n_added [n_tc]: 0, 1 or 2 MDs; t3 [n_tc]: index of the triplet used in the
 * stage-2 object list (-1: none); attrs [n_tc x 3]: chi2_xy, chi2_rz and
 * curvature of the extended chain (zeros: none).  Any array may be NULL.
 * Errors: LST_E_STATE if the event failed, is not complete, or was enqueued
 * while the extensions were disabled. */
lst_status lst_get_extended_track_candidates(lst_event ev, int32_t *n_tc, int32_t *n_hits_total, int32_t *type,
                                             int32_t *offsets, int32_t *hits, int32_t *n_added, int32_t *t3,
                                             float *attrs);

/* Objects of one stage, copied to HOST buffers (two-call protocol as above;
 * NULL arrays to query *n).  tuples [n x w] with w = 2, 4, 6, 10, 1, 7, 11 for
 * stages 0..6: hit indices of the MDs inner to outer (lower, upper), with the
 * seed index first for pLS/pT3/pT5.  flags [n]: 1 if the object survives
 * duplicate removal (T5, pLS, pT3, pT5), else 1.  attrs [n x a] with a = 0, 2,
 * 4, 8, 5, 3, 3:  LS beta_in, beta_out;  T3 kappa, dkappa, chi2_rz, lambda;
 * T5 kappa, chi2_xy, chi2_rz, lambda, kappa_in, kappa_out, dir_x, dir_y;
 * pLS pT, cos, sin, lambda, kappa;  pT3/pT5 chi2_xy, chi2_rz, score. */
lst_status lst_get_stage_objects(lst_event ev, int32_t stage, int32_t *n, int32_t *tuples, int32_t *flags,
                                 float *attrs);

/* counts[0..7]: object counts per stage (MD .. TC) as built; required[0..7]:
 * counts that would have been built without capacity limits (equal to
 * counts unless the status was LST_E_CAPACITY).  Either may be NULL. */
lst_status lst_get_stage_counts(lst_event ev, int64_t *counts, int64_t *required);

/* Per-module mini-doublet window constants as uploaded (4 floats per module:
 * W, A1, A2, A3), copied to a HOST buffer of 4 * n_modules floats. */
lst_status lst_get_module_constants(lst_geometry geom, float *out);

/* Live timing of one kernel launch site (for roofline measurement).  The
 * chain is a fixed sequence of launch sites, each launched once per event:
 * lst_kernel_site_count() of them, named by lst_kernel_site_name(i) (NULL
 * for an invalid index).  lst_set_timed_site(i) makes every later enqueue in
 * the process bracket site i with two HIP events on the event's stream (-1 =
 * off); lst_get_site_time() returns that site's duration in milliseconds for
 * a completed event (LST_E_STATE if no site was timed). */
int32_t lst_kernel_site_count(void);
const char *lst_kernel_site_name(int32_t site);
lst_status lst_set_timed_site(int32_t site);
lst_status lst_get_site_time(lst_event ev, float *ms);

/* Launch shapes and autotuning.  Some launch sites (the segment, triplet,
 * quintuplet, pixel-seed and cleaning searches) accept a block of 64, 128 or
 * 256 threads; the geometry holds one choice per site and every later
 * enqueue, batch, plan capture and server launch on that geometry uses it.
 * Results do not depend on the choice.  Arrays have lst_kernel_site_count()
 * entries, indexed by launch site.
 *  lst_get_launch_config: threads per block of each tunable site, 0 for the
 *    sites with a fixed shape.
 *  lst_set_launch_config: 0 (default, 256), 64, 128 or 256 for a tunable site,
 *    0 for the others; LST_E_INVALID otherwise (nothing is changed).
 *  lst_autotune: runs the caller's B events (device descriptors, as
 *    lst_enqueue_batch, in `workspace` of lst_batch_workspace_bytes() bytes)
 *    reps times per choice of each tunable site in turn, timing that site with
 *    HIP events on `stream`, keeps the fastest choice per site and returns in
 *    site_ms (optional) the best time of each tuned site (-1 for the others).
 *    It waits for the device; on any error the previous shapes are restored.
 *    Not to be called while other calls use the same geometry. */
lst_status lst_get_launch_config(lst_geometry geom, int32_t n, int32_t *site_block);
lst_status lst_set_launch_config(lst_geometry geom, int32_t n, const int32_t *site_block);
lst_status lst_autotune(lst_geometry geom, int32_t B, const lst_event_desc *evs, const lst_capacity *cap,
                        void *workspace, size_t ws_bytes, void *stream, int32_t reps, float *site_ms);

/* Tile choices of the chain, per geometry (applied to chains enqueued and
 * plans created afterwards; results do not depend on them).  Tile i in
 * [0, lst_tile_count()) is named by lst_tile_name(i):
 *   md_cache, ls_cache, t3_cache, t5_cache: passing partners per parent that
 *     the MD / segment / triplet / quintuplet count pass remembers (module,
 *     MD, segment, triplet), so that its fill copies them instead of
 *     searching again (a parent with more is searched again);
 *   pt3_cache, pt5_cache: pT3 / pT5 per seed the seed-search count keeps with
 *     their attributes (Section 2.4);
 *   pass_list: passing objects of one seed ranked in on-chip memory by the
 *     seed-search fill (a seed with more is filled by an ordered scan of all
 *     objects);
 *   max_slices: marked (ring, azimuth) bins of one seed gathered into one flat
 *     candidate list (more: searched bin by bin);
 *   ext_per_wave: track candidates per wavefront of the extension search
 *     (4, 8 or 16);
 *   ls_group: inner MDs per wavefront of the segment count pass (1..16),
 *     whose selections share full wavefronts; 0 (the default) chooses per
 *     launch from its events and MD capacity (4 for one PU200-size event, 16
 *     for launches of 16 or more).
 * lst_tile_range gives tile i's bounds; lst_get/set_tile_config read and
 * write all lst_tile_count() values at once (LST_E_INVALID and nothing changed
 * if one is out of range).  lst_autotune_tiles times the whole chain over the
 * caller's B events (as lst_autotune) for each candidate value of each tile
 * in turn, keeps the fastest, and returns in tile_ms (optional,
 * lst_tile_count() entries) the best chain time per tile (-1 for tiles not
 * tuned: ext_per_wave without track extensions).  It waits for the device;
 * on error the previous tiles are restored.  Not to be called while other
 * calls use the same geometry. */
int32_t lst_tile_count(void);
const char *lst_tile_name(int32_t i);
lst_status lst_tile_range(int32_t i, int32_t *lo, int32_t *hi);
lst_status lst_get_tile_config(lst_geometry geom, int32_t n, int32_t *tiles);
lst_status lst_set_tile_config(lst_geometry geom, int32_t n, const int32_t *tiles);
lst_status lst_autotune_tiles(lst_geometry geom, int32_t B, const lst_event_desc *evs, const lst_capacity *cap,
                              void *workspace, size_t ws_bytes, void *stream, int32_t reps, float *tile_ms);

/* Counter calibration: launches n_blocks groups of 256 threads that each run
 * `iters` rounds of 16 independent fused multiply-adds (no memory traffic;
 * `out`, n_blocks * 256 floats of DEVICE memory, is never written in
 * practice), on `stream`, without waiting.  Its known instruction count and
 * stall-free issue calibrate the vector-issue counters that the profile
 * summaries report for the chain's kernels.  LST_E_INVALID for bad arguments,
 * LST_E_DEVICE if the launch fails. */
lst_status lst_probe_valu(int32_t n_blocks, int32_t iters, float *out, void *stream);

lst_status lst_release_event(lst_event ev);
const char *lst_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LST_H */
