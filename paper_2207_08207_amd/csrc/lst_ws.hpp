// Workspace layout and launch interface of the LST chain (host + device).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lst {

// Counter slots (int32) at the start of the workspace.
enum Ctr : int {
  C_STATUS = 0,  // bit 0: invalid hit data, bit 1: invalid seed data, bit 2: capacity exceeded
  C_NMD = 1, C_NLS, C_NT3, C_NT5, C_NPT3, C_NPT5, C_NTC, C_NTCHITS,   // built counts (clamped)
  C_RMD = 9, C_RLS, C_RT3, C_RT5, C_RPT3, C_RPT5,                      // required counts
  C_NT5KEEP = 15, C_NTC0 = 16, C_NTC1, C_NTC2, C_NTC3,                 // survivors, TCs per type
  C_NOUTER = 20, C_NINC = 21, C_NPH = 22, C_NO3 = 23, C_NO5 = 24,      // scratch totals
  C_NB3 = 25, C_NB5 = 26,
  C_NLSOVF = 27,                 // MDs with more segments than the count pass caches
  C_NEXTHITS = 28,               // hits of the extended track-candidate collection
  C_EXT = 29,                    // 1 once the track extensions of the event are written
  C_NDENSE = 30,                 // modules with more than kMdBig hit pairs (listed in md_dense)
  C_COUNT = 64
};
enum : int { ST_BAD_HIT = 1, ST_BAD_SEED = 2, ST_CAPACITY = 4 };

// Tile choices of the chain, set per geometry at run time (lst_set_tile_config,
// lst_autotune): how many passing partners a count pass remembers per parent
// (its fill copies them instead of searching again), the seed search's LDS
// list and slice table, and the candidates per wave of the extension search.
// Storage and LDS arrays are sized for the maxima (the kXxx constants below);
// results never depend on the choice.
struct Tiles {
  int md_cache;      // MDs per module whose (lower, upper) pair the MD count pass keeps, 0..kMdCache
  int ls_cache;      // segments per MD the segment count pass keeps, 0..kLsCache
  int t3_cache;      // triplets per segment the triplet count pass keeps, 0..kT3Cache
  int t5_cache;      // quintuplets per triplet the quintuplet count pass keeps, 0..kT5Cache
  int pt3_cache;     // pT3 per seed the seed-search count keeps with attributes, 0..kPt3Cache
  int pt5_cache;     // pT5 per seed, 0..kPt5Cache
  int pass_list;     // passing objects per seed ranked in LDS by the fill, 1..kPassList (else: ordered scan)
  int max_slices;    // marked bins per seed gathered into one flat list, 1..kMaxSlices (else: bin by bin)
  int ext_per_wave;  // track candidates per wave of the extension search: 4, 8 or 16
  int ls_group;      // inner MDs per wave of the segment count pass, 1..kLsGroup; 0: chosen per launch
};

struct DevGeom {
  int n_mod, n_edges;
  const int *map_off, *map_tgt;
  const float4 *win;  // per module: W, A1, A2, A3
  const int *info;    // per module: bit 0 = 2S, bit 1 = endcap
  int ext;            // 1: the chain ends with the track extensions
  float d0max;        // transverse impact-parameter bound of the selections [cm]
  int stub16;         // 1: MD stubs stored as binary16 pairs (dense half2), else float2
  const float2 *t5cut;  // per quintuplet category (1024): chi2_xy and chi2_rz bounds
  Tiles tiles;
};

// One exclusive scan of the chain: out[0..n] = scan of in[0..n), n = *n_dev
// (or n_fix); the total goes to *tot_req and, clamped to cap (overflow
// flagged), to *tot_clamped.  n_cap bounds n for the launch grid.
struct ScanJob {
  const int *in;
  int *out;
  const int *n_dev;
  int n_fix, n_cap;
  int *tot_req, *tot_clamped;
  int cap;
};
enum ScanId : int {
  SC_HITS, SC_MD, SC_LS, SC_T3, SC_T5, SC_INC, SC_PH, SC_PT3, SC_PT5,
  SC_F5, SC_F3, SC_FT5, SC_FPLS, SC_B3, SC_B5, SC_LSOVF, SC_EXT, SC_COUNT
};
// One array cleared to zero at the start of the chain.
// n: the array's length; with n_dev, only its first mul * (*n_dev + 1)
// entries (the device-side count of what it is indexed by, plus one) when
// that is fewer.
struct FillJob {
  int *p;
  long n;
  const int *n_dev;
  int mul;
};
enum FillId : int {
  FL_CTR, FL_INC_CNT, FL_INC_CUR, FL_PH_CNT, FL_PH_CUR, FL_O3_BEST,
  FL_O5_BEST, FL_SEED_USED, FL_T5_USED, FL_B3_CNT, FL_B3_CUR, FL_B5_CNT, FL_B5_CUR, FL_COUNT
};

// Passing partners remembered between a stage's count and fill passes: per
// module for mini-doublets, per MD for segments, per seed for pT3 / pT5 (more
// than this: the fill searches again).
constexpr int kLsCache = 32;
constexpr int kLsGroup = 16;  // most inner MDs per wave of the segment count pass
constexpr int kMdCache = 32;  // MDs per module whose (lower, upper) pair the MD count pass keeps
constexpr int kMdParts = 16;   // waves of a dense module's block (k_md_big), one part of its pairs each
constexpr int kMdQCache = 16;  // MDs per part of a dense module whose pair the MD count pass keeps
constexpr int kT3Cache = 2;   // triplets per parent segment whose candidate the T3 count pass keeps
constexpr int kT5Cache = 2;   // quintuplets per parent triplet whose candidate the T5 count pass keeps
constexpr int kPt3Cache = 256;  // pT3 per seed (PU200 maximum ~190)
constexpr int kPt5Cache = 16;   // pT5 per seed
// Hit bucketing: block tiles of kHitTile input hits (four waves of 1024);
// (module, sensor) keys in coarse buckets of kFineKeys consecutive keys (at
// most kMaxCoarse of them, so 2 n_mod <= kFineKeys * kMaxCoarse).
constexpr int kHitTile = 4096;
constexpr int kFineBits = 5, kFineKeys = 1 << kFineBits;
constexpr int kMaxCoarse = 2048;
constexpr int kMaxModules = kFineKeys * kMaxCoarse / 2;
__host__ __device__ inline int n_coarse(int n_mod) { return (2 * n_mod + kFineKeys - 1) / kFineKeys; }
__host__ __device__ inline int n_hit_tiles(long n_hits) { return (int)((n_hits + kHitTile - 1) / kHitTile); }
constexpr int kPassList = 1024;  // passing objects of one seed ranked in LDS by the seed-search fill
constexpr int kMaxSlices = 512;  // marked bins of one seed gathered into a flat list in LDS
constexpr int kExtPerWaveMax = 16;
constexpr Tiles kTilesDefault{kMdCache, kLsCache, kT3Cache, kT5Cache, kPt3Cache, kPt5Cache, kPassList, kMaxSlices, 8, 0};

// First-anchor bins of the seed search: 10 radius rings x 256 azimuth bins x
// 55 z bins (10 cm over |z| < 275 cm); bins of one (ring, azimuth) pair are
// contiguous, z ascending.
constexpr int kSeedBins = 10 * 256 * 55;

// Device pointers of one event (all inside the workspace except the inputs).
// Kernels of a batch read descriptor blockIdx.y of a device array of these.
struct Ws {
  // inputs (device)
  int n_hits, n_seeds;
  const float *x, *y, *z, *px, *py, *pz;
  const int *module, *sensor, *q, *hits4;
  // capacities
  int cap_md, cap_ls, cap_t3, cap_t5, cap_pt3, cap_pt5, cap_tc;
  int *ctr;
  // hit buckets by (module, sensor)
  int *boff, *hidx;  // (module, sensor) buckets: offsets (2 n_mod + 1), input index per bucketed hit
  int *tile_hist, *tile_off;  // hits per (coarse bucket, wave tile), coarse-bucket major, and their scan
  float4 *hcp;  // hits in coarse-bucket order (stable): x, y, z, input index | key within the bucket << 23 (bits)
  float4 *hpos;
  // mini-doublets
  int *md_cnt, *md_off;
  int *md_cache;     // per module: up to kMdCache passing pairs (lower << 16 | upper) of the count pass
  int *md_part;      // per dense module: MDs of each wave's part of its pairs (count pass)
  int *md_bcache;    // per dense module and part: up to kMdQCache passing pairs (lower << 16 | upper)
  int *md_dense;     // the dense modules, listed (in any order) by the small-module MD count pass
  int2 *md_hits;    // input indices of the lower and upper hit
  int *md_mod;
  float4 *md_pos;   // anchor (lower hit) x, y, z, r
  float2 *md_stub;  // tangential displacement, sensor separation (dense half2 with DevGeom::stub16)
  float4 *mod_disc;  // per module with MDs: x-y disc (cx, cy, radius, |c|) around its anchors
  // segments
  int *ls_cnt, *ls_off;
  int *ls_cache;    // per MD: up to kLsCache passing partners found by the count pass (| info << 30)
  int *ls_ovf_flag, *ls_ovf_off, *ls_ovf;  // MDs with more: flag, its scan, the dense list
  int2 *ls_md;
  float2 *ls_beta;
  float4 *ls_opos;  // the outer MD's anchor (a copy, read by the triplet search)
  int *ls_oinf;      // and its module's info word
  // triplets
  int *t3_cnt, *t3_off;
  int4 *t3_md;      // a, b, c, -
  float4 *t3_attr;  // kappa, dkappa, chi2_rz, lambda
  float2 *t3_first; // anchor x, y of the first MD
  int *t3_cache;    // per segment: up to kT3Cache passing candidate segments of the count pass
  // quintuplets
  int *t5_cnt, *t5_off;
  int2 *t5_t3;
  int *t5_md;       // 5 per T5
  float *t5_attr;   // 8 per T5
  int *t5_keep;
  float2 *t5_first;
  int *t5_cache;    // per triplet: up to kT5Cache passing candidate triplets of the count pass
  int *inc_cnt, *inc_off, *inc_cur;
  int2 *inc_list;   // T5s containing each MD: (T5, bits of its chi2_xy score)
  // pixel seeds
  float *pls;       // 8 per seed: pT, cx, cy, lambda, kappa, x0, y0, z0
  int *pls_keep;
  int *seed_order;  // seeds in the seed search's processing order (grouped by direction)
  int *ph_cnt, *ph_off, *ph_cur, *ph_list;      // seeds using each pixel hit
  // pixel triplets / quintuplets
  int *pt3_cnt, *pt3_off, *pt5_cnt, *pt5_off;
  int *pt3_cache, *pt5_cache;  // per seed: up to kPt3Cache / kPt5Cache passing objects found by the count pass
  float4 *pt3_cattr, *pt5_cattr;  // and their attributes
  int2 *pt3_so, *pt5_so;      // seed, object
  float4 *pt3_attr, *pt5_attr;
  int *pt3_keep, *pt5_keep;
  // per T3 / T5: the largest ~(score bits << 32 | seed) of the pT3 / pT5 entries on it,
  // i.e. its entry with the smallest (score, seed) (scores are >= 0, so their bits order them)
  unsigned long long *o3_best, *o5_best;
  int *b3_cnt, *b3_off, *b3_cur, *b3_list;      // T3s by first-anchor (ring, azimuth, z) bin
  int *b5_cnt, *b5_off, *b5_cur, *b5_list;      // surviving T5s by the same bins
  float4 *b3_pos, *b5_pos;  // per list entry: the object's first anchor x, y, z and module info bits
  // track candidates
  int *seed_used, *t5_used;
  int *f_pt5, *f_pt3, *f_t5, *f_pls;            // TC flags
  int *p_pt5, *p_pt3, *p_t5, *p_pls;            // their exclusive scans
  float4 *dir_pt5, *dir_pt3, *dir_t5;           // compact directions (dx, dy, lambda)
  float4 *bdir_pt5, *bdir_pt3, *bdir_t5;        // the same, grouped by azimuth bin
  int *boff_pt5, *boff_pt3, *boff_t5;           // bin offsets (kDirBins + 1)
  int *tc_type, *tc_off, *tc_hits;
  int *tc_md;                                   // its outer-tracker MDs, inner to outer (5 per TC)
  float2 *tc_kap;                               // its curvature and curvature tolerance
  // track extensions, per TC: MDs added (0-2), triplet (-1: none), (chi2_xy, chi2_rz, kappa),
  // hit count of the extended TC, its exclusive scan, the extended hit lists
  int *ext_n, *ext_t3, *ext_cnt, *ext_off, *ext_hits;
  float4 *ext_attr;
  // scan scratch and the job tables of the generic scan / clear kernels
  int *scan_tmp;
  ScanJob scans[SC_COUNT];
  FillJob fills[FL_COUNT];
};

// Capacities and sizes (host-side).
struct Caps {
  int64_t md, ls, t3, t5, pt3, pt5;
};

// Carves one event's arrays from `base` (nullptr: size only) and fills the
// scan / clear job tables; counters go to `ctr` (64 ints) when given.
// Array sizes follow n_hits_alloc / n_seeds_alloc when those are >= 0 (a
// slot of a captured plan is sized for the largest event it may hold).
size_t workspace_layout(int n_mod, int n_hits, int n_seeds, const Caps &c, Ws *ws, char *base, int *ctr,
                        int n_hits_alloc = -1, int n_seeds_alloc = -1);
// Brackets launch site `site` of the chain with two recorded HIP events.
struct KernelTimer {
  int site;
  hipEvent_t beg, end;
};
constexpr int kChainSite = 1000;  // KernelTimer::site that brackets the whole chain
extern const char *const kSiteNames[];
extern const int kNumSites;
constexpr int kMaxSites = 64;
// True for the launch sites that take a block of 64, 128 or 256 threads.
bool site_tunable(int site);
// Enqueues the whole chain for B events whose descriptors are d_ws[0..B) in
// device memory; `bound` holds, field by field, the largest sizes and
// capacities of the batch (it sets the launch grids).  site_block (kMaxSites
// entries or NULL): threads per block of each tunable site, 0 = the default.
void enqueue_chain(const DevGeom &g, const Ws *d_ws, int B, const Ws &bound, hipStream_t st, const KernelTimer *kt,
                   const int *site_block);
void launch_module_windows(const int *info, const float *pos_lo, const float *pos_up, const float *lmin,
                           const float *lmax, int n_mod, double d0, float4 *win, hipStream_t st);
// Allocation-free forms: an event descriptor written by a kernel, and the
// track candidates copied to caller device buffers (counts: n, hits, status).
void launch_put_desc(const Ws &w, Ws *dst, hipStream_t st);
void launch_tc_export(const Ws *d_ws, int max_tc, int max_hits, int *type, int *off, int *hits, int *counts,
                      hipStream_t st);

}  // namespace lst
