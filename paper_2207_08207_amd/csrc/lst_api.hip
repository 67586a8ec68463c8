// C ABI of the LST library (include/lst.h): argument checks, geometry upload,
// workspace carving, enqueue of the kernel chain, result copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <atomic>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lst.h"
#include "lst_ws.hpp"

namespace {

thread_local std::string g_err;

lst_status fail(lst_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                               \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return fail(LST_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kTupleW[7] = {2, 4, 6, 10, 1, 7, 11};
constexpr int kAttrW[7] = {0, 2, 4, 8, 5, 3, 3};
constexpr int64_t kMaxCap = 8000000;  // bounded by the two-level device scan (4096 x 2048)
std::atomic<int> g_timed_site{-1};

}  // namespace

struct lst_geometry_s {
  lst::DevGeom g;
  int *d_off = nullptr, *d_tgt = nullptr, *d_info = nullptr;
  float4 *d_win = nullptr;
};

struct lst_event_s {
  lst_geometry geom = nullptr;
  lst::Ws ws{};
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int *h_ctr = nullptr;  // pinned copy of the counters
  bool synced = false;
  int timed_site = -1;   // launch site bracketed by beg/end, or -1
  hipEvent_t tbeg = nullptr, tend = nullptr;
  lst_status status = LST_OK;
};

namespace lst {

size_t workspace_layout(int n_mod, int n_hits, int n_seeds, const Caps &c, Ws *w, char *base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    off = (off + kAlign - 1) / kAlign * kAlign;
    char *p = base ? base + off : nullptr;
    off += bytes ? bytes : 1;
    return p;
  };
  const long N = n_hits, S = n_seeds, M = n_mod;
  const long md = c.md, ls = c.ls, t3 = c.t3, t5 = c.t5, p3 = c.pt3, p5 = c.pt5;
  const long tc = p5 + p3 + t5 + S;
#define I(n) reinterpret_cast<int *>(take(sizeof(int) * (size_t)(n)))
#define F(n) reinterpret_cast<float *>(take(sizeof(float) * (size_t)(n)))
#define I2(n) reinterpret_cast<int2 *>(take(sizeof(int2) * (size_t)(n)))
#define I4(n) reinterpret_cast<int4 *>(take(sizeof(int4) * (size_t)(n)))
#define F2(n) reinterpret_cast<float2 *>(take(sizeof(float2) * (size_t)(n)))
#define F4(n) reinterpret_cast<float4 *>(take(sizeof(float4) * (size_t)(n)))
  Ws t{};
  t.ctr = I(C_COUNT);
  t.bcnt = I(2 * M + 1); t.boff = I(2 * M + 1); t.bcur = I(2 * M);
  t.hidx_tmp = I(N + 1); t.hidx = I(N + 1); t.hpos = F4(N + 1);
  t.md_cnt = I(M + 1); t.md_off = I(M + 1);
  t.md_hits = I2(md); t.md_mod = I(md); t.md_pos = F4(md); t.md_stub = F2(md);
  t.ls_cnt = I(md + 1); t.ls_off = I(md + 1); t.ls_md = I2(ls); t.ls_beta = F2(ls);
  t.t3_cnt = I(ls + 1); t.t3_off = I(ls + 1); t.t3_md = I4(t3); t.t3_attr = F4(t3); t.t3_first = F2(t3);
  t.t5_cnt = I(t3 + 1); t.t5_off = I(t3 + 1); t.t5_t3 = I2(t5); t.t5_md = I(5 * t5); t.t5_attr = F(8 * t5);
  t.t5_keep = I(t5); t.t5_first = F2(t5);
  t.inc_cnt = I(md + 1); t.inc_off = I(md + 1); t.inc_cur = I(md + 1); t.inc_list = I(5 * t5);
  t.pls = F(8 * S); t.pls_keep = I(S);
  t.ph_cnt = I(N + 1); t.ph_off = I(N + 1); t.ph_cur = I(N + 1); t.ph_list = I(4 * S);
  t.pt3_cnt = I(S + 1); t.pt3_off = I(S + 1); t.pt5_cnt = I(S + 1); t.pt5_off = I(S + 1);
  t.pt3_so = I2(p3); t.pt5_so = I2(p5); t.pt3_attr = F4(p3); t.pt5_attr = F4(p5);
  t.pt3_keep = I(p3); t.pt5_keep = I(p5);
  t.o3_cnt = I(t3 + 1); t.o3_off = I(t3 + 1); t.o3_cur = I(t3 + 1); t.o3_list = I(p3);
  t.o5_cnt = I(t5 + 1); t.o5_off = I(t5 + 1); t.o5_cur = I(t5 + 1); t.o5_list = I(p5);
  t.seed_used = I(S + 1); t.t5_used = I(t5 + 1);
  t.f_pt5 = I(p5 + 1); t.f_pt3 = I(p3 + 1); t.f_t5 = I(t5 + 1); t.f_pls = I(S + 1);
  t.p_pt5 = I(p5 + 1); t.p_pt3 = I(p3 + 1); t.p_t5 = I(t5 + 1); t.p_pls = I(S + 1);
  t.dir_pt5 = F4(p5); t.dir_pt3 = F4(p3); t.dir_t5 = F4(t5);
  t.bdir_pt5 = F4(p5); t.bdir_pt3 = F4(p3); t.bdir_t5 = F4(t5);
  t.boff_pt5 = I(129); t.boff_pt3 = I(129); t.boff_t5 = I(129);
  t.tc_type = I(tc); t.tc_off = I(tc + 1); t.tc_hits = I(14 * tc);
  t.scan_tmp = I(4096);
#undef I
#undef F
#undef I2
#undef I4
#undef F2
#undef F4
  t.cap_md = (int)md; t.cap_ls = (int)ls; t.cap_t3 = (int)t3; t.cap_t5 = (int)t5;
  t.cap_pt3 = (int)p3; t.cap_pt5 = (int)p5; t.cap_tc = (int)tc;
  t.n_hits = n_hits; t.n_seeds = n_seeds;
  if (w) *w = t;
  return (off + kAlign - 1) / kAlign * kAlign;
}

}  // namespace lst

template <typename T>
static hipError_t d2h(std::vector<T> &v, const void *src, size_t n) {
  v.resize(n ? n : 1);
  if (!n) return hipSuccess;
  return hipMemcpy(v.data(), src, sizeof(T) * n, hipMemcpyDeviceToHost);
}

static void drop(hipError_t) {}

static lst_status check_caps(const lst_capacity &c) {
  const int64_t v[6] = {c.md, c.ls, c.t3, c.t5, c.pt3, c.pt5};
  for (int i = 0; i < 6; ++i)
    if (v[i] < 1 || v[i] > kMaxCap) return fail(LST_E_INVALID, "capacity out of range [1, 8e6]");
  return LST_OK;
}

extern "C" {

const char *lst_last_error(void) { return g_err.c_str(); }

lst_status lst_default_capacity(int32_t n_hits, int32_t n_seeds, lst_capacity *out) {
  if (!out || n_hits < 0 || n_seeds < 0) return fail(LST_E_INVALID, "lst_default_capacity: bad argument");
  const int64_t N = n_hits, S = n_seeds;
  auto clampc = [](int64_t v) { return v < 1024 ? (int64_t)1024 : (v > kMaxCap ? kMaxCap : v); };
  out->md = clampc(N);
  out->ls = clampc(4 * N);
  out->t3 = clampc(2 * N);
  out->t5 = clampc(N);
  out->pt3 = clampc(64 * S);
  out->pt5 = clampc(16 * S);
  return LST_OK;
}

lst_status lst_load_geometry(const lst_geometry_desc *d, lst_geometry *out) {
  if (!d || !out) return fail(LST_E_INVALID, "lst_load_geometry: NULL argument");
  *out = nullptr;
  const int M = d->n_modules, E = d->n_edges;
  if (M <= 0 || E < 0 || !d->subdet || !d->type || !d->pos_lo || !d->pos_up || !d->lmin || !d->lmax ||
      !d->map_offsets || (E > 0 && !d->map_targets))
    return fail(LST_E_INVALID, "lst_load_geometry: missing array or bad size");
  if (d->map_offsets[0] != 0 || d->map_offsets[M] != E)
    return fail(LST_E_INVALID, "lst_load_geometry: map_offsets must start at 0 and end at n_edges");
  for (int m = 0; m < M; ++m) {
    if (d->map_offsets[m + 1] < d->map_offsets[m]) return fail(LST_E_INVALID, "map_offsets not monotone");
    if ((d->subdet[m] != 0 && d->subdet[m] != 1) || (d->type[m] != 0 && d->type[m] != 1))
      return fail(LST_E_INVALID, "subdet/type must be 0 or 1");
    if (!(d->pos_lo[m] > 0.0f) || !(d->pos_up[m] > d->pos_lo[m]) || !(d->lmax[m] > d->lmin[m]))
      return fail(LST_E_INVALID, "module sensor positions or long range invalid");
    if (d->subdet[m] == 1 && !(d->pos_lo[m] > 20.0f)) return fail(LST_E_INVALID, "endcap sensor too close to z = 0");
  }
  for (int e = 0; e < E; ++e)
    if (d->map_targets[e] < 0 || d->map_targets[e] >= M) return fail(LST_E_INVALID, "map target out of range");
  for (int m = 0; m < M; ++m)
    if (d->map_offsets[m + 1] - d->map_offsets[m] > 256)
      return fail(LST_E_INVALID, "more than 256 module-map targets for one module");
  auto *g = new (std::nothrow) lst_geometry_s();
  if (!g) return fail(LST_E_NOMEM, "host allocation failed");
  std::vector<int> info(M);
  for (int m = 0; m < M; ++m) info[m] = (d->type[m] & 1) | ((d->subdet[m] & 1) << 1);
  float *d_pos = nullptr;
  auto cleanup = [&]() {
    drop(hipFree(g->d_off)); drop(hipFree(g->d_tgt)); drop(hipFree(g->d_info)); drop(hipFree(g->d_win));
    drop(hipFree(d_pos));
    delete g;
  };
  if (hipMalloc(&g->d_off, sizeof(int) * (M + 1)) != hipSuccess ||
      hipMalloc(&g->d_tgt, sizeof(int) * (E > 0 ? E : 1)) != hipSuccess ||
      hipMalloc(&g->d_info, sizeof(int) * M) != hipSuccess || hipMalloc(&g->d_win, sizeof(float4) * M) != hipSuccess ||
      hipMalloc(&d_pos, sizeof(float) * 4 * M) != hipSuccess) {
    cleanup();
    return fail(LST_E_NOMEM, "lst_load_geometry: device allocation failed");
  }
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemcpy(g->d_off, d->map_offsets, sizeof(int) * (M + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && E > 0) e = hipMemcpy(g->d_tgt, d->map_targets, sizeof(int) * E, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(g->d_info, info.data(), sizeof(int) * M, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_pos, d->pos_lo, sizeof(float) * M, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_pos + M, d->pos_up, sizeof(float) * M, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_pos + 2 * M, d->lmin, sizeof(float) * M, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_pos + 3 * M, d->lmax, sizeof(float) * M, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    lst::launch_module_windows(g->d_info, d_pos, d_pos + M, d_pos + 2 * M, d_pos + 3 * M, M, g->d_win, nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    cleanup();
    return fail(LST_E_DEVICE, std::string("lst_load_geometry: ") + hipGetErrorString(e));
  }
  drop(hipFree(d_pos));
  g->g.n_mod = M;
  g->g.n_edges = E;
  g->g.map_off = g->d_off;
  g->g.map_tgt = g->d_tgt;
  g->g.win = g->d_win;
  g->g.info = g->d_info;
  *out = g;
  return LST_OK;
}

lst_status lst_release_geometry(lst_geometry g) {
  if (!g) return LST_OK;
  drop(hipFree(g->d_off)); drop(hipFree(g->d_tgt)); drop(hipFree(g->d_info)); drop(hipFree(g->d_win));
  delete g;
  return LST_OK;
}

lst_status lst_get_module_constants(lst_geometry g, float *out) {
  if (!g || !out) return fail(LST_E_INVALID, "lst_get_module_constants: NULL argument");
  HIP_TRY(hipMemcpy(out, g->d_win, sizeof(float4) * g->g.n_mod, hipMemcpyDeviceToHost));
  return LST_OK;
}

lst_status lst_workspace_bytes(lst_geometry g, int32_t n_hits, int32_t n_seeds, const lst_capacity *cap,
                               size_t *bytes) {
  if (!g || !bytes || n_hits < 0 || n_seeds < 0 || n_hits > kMaxCap || n_seeds > kMaxCap / 4)
    return fail(LST_E_INVALID, "lst_workspace_bytes: bad argument");
  lst_capacity c;
  if (cap) c = *cap; else lst_default_capacity(n_hits, n_seeds, &c);
  lst_status s = check_caps(c);
  if (s != LST_OK) return s;
  lst::Caps cc{c.md, c.ls, c.t3, c.t5, c.pt3, c.pt5};
  *bytes = lst::workspace_layout(g->g.n_mod, n_hits, n_seeds, cc, nullptr, nullptr);
  return LST_OK;
}

static lst_status map_status(int st) {
  if (st & (lst::ST_BAD_HIT | lst::ST_BAD_SEED))
    return fail(LST_E_INVALID, (st & lst::ST_BAD_HIT) ? "invalid hit data (module/sensor out of range or non-finite)"
                                                      : "invalid seed data (hit index, charge or momentum)");
  if (st & lst::ST_CAPACITY) return fail(LST_E_CAPACITY, "object capacity exceeded; see lst_get_stage_counts");
  return LST_OK;
}

lst_status lst_enqueue_event(lst_geometry g, const lst_event_desc *ev, const lst_capacity *cap, void *workspace,
                             size_t ws_bytes, void *stream, lst_event *out) {
  if (!out) return fail(LST_E_INVALID, "lst_enqueue_event: NULL out");
  *out = nullptr;
  if (!g || !ev || !workspace) return fail(LST_E_INVALID, "lst_enqueue_event: NULL argument");
  if (ev->n_hits < 0 || ev->n_seeds < 0) return fail(LST_E_INVALID, "negative n_hits or n_seeds");
  if (ev->n_hits > kMaxCap || ev->n_seeds > kMaxCap / 4) return fail(LST_E_INVALID, "n_hits above 8e6 or n_seeds above 2e6");
  if (ev->n_hits > 0 && (!ev->x || !ev->y || !ev->z || !ev->module || !ev->sensor))
    return fail(LST_E_INVALID, "hit arrays missing");
  if (ev->n_seeds > 0 && (!ev->px || !ev->py || !ev->pz || !ev->q || !ev->hits4))
    return fail(LST_E_INVALID, "seed arrays missing");
  if (ev->n_seeds > 0 && ev->n_hits == 0) return fail(LST_E_INVALID, "seeds without hits");
  lst_capacity c;
  if (cap) c = *cap; else lst_default_capacity(ev->n_hits, ev->n_seeds, &c);
  lst_status s = check_caps(c);
  if (s != LST_OK) return s;
  lst::Caps cc{c.md, c.ls, c.t3, c.t5, c.pt3, c.pt5};
  const size_t need = lst::workspace_layout(g->g.n_mod, ev->n_hits, ev->n_seeds, cc, nullptr, nullptr);
  if (ws_bytes < need)
    return fail(LST_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return fail(LST_E_INVALID, "workspace not 256-byte aligned");
  auto *e = new (std::nothrow) lst_event_s();
  if (!e) return fail(LST_E_NOMEM, "host allocation failed");
  e->geom = g;
  e->stream = reinterpret_cast<hipStream_t>(stream);
  lst::workspace_layout(g->g.n_mod, ev->n_hits, ev->n_seeds, cc, &e->ws, reinterpret_cast<char *>(workspace));
  lst::Ws &w = e->ws;
  w.x = ev->x; w.y = ev->y; w.z = ev->z; w.module = ev->module; w.sensor = ev->sensor;
  w.px = ev->px; w.py = ev->py; w.pz = ev->pz; w.q = ev->q; w.hits4 = ev->hits4;
  if (hipHostMalloc(reinterpret_cast<void **>(&e->h_ctr), sizeof(int) * lst::C_COUNT, hipHostMallocDefault) !=
          hipSuccess ||
      hipEventCreateWithFlags(&e->done, hipEventDisableTiming) != hipSuccess) {
    if (e->h_ctr) drop(hipHostFree(e->h_ctr));
    delete e;
    return fail(LST_E_DEVICE, "lst_enqueue_event: pinned buffer or event creation failed");
  }
  lst::KernelTimer kt{-1, nullptr, nullptr};
  const int site = g_timed_site.load();
  if (site >= 0 && hipEventCreate(&e->tbeg) == hipSuccess && hipEventCreate(&e->tend) == hipSuccess) {
    kt = lst::KernelTimer{site, e->tbeg, e->tend};
    e->timed_site = site;
  }
  lst::enqueue_chain(g->g, w, e->stream, e->timed_site >= 0 ? &kt : nullptr);
  hipError_t he = hipGetLastError();
  if (he == hipSuccess)
    he = hipMemcpyAsync(e->h_ctr, w.ctr, sizeof(int) * lst::C_COUNT, hipMemcpyDeviceToHost, e->stream);
  if (he == hipSuccess) he = hipEventRecord(e->done, e->stream);
  if (he != hipSuccess) {
    e->status = LST_E_DEVICE;
    *out = e;
    return fail(LST_E_DEVICE, std::string("lst_enqueue_event: ") + hipGetErrorString(he));
  }
  *out = e;
  return LST_OK;
}

lst_status lst_event_query(lst_event e, int32_t *done) {
  if (!e || !done) return fail(LST_E_INVALID, "lst_event_query: NULL argument");
  if (e->synced) { *done = 1; return LST_OK; }
  hipError_t q = hipEventQuery(e->done);
  if (q == hipErrorNotReady) { *done = 0; return LST_OK; }
  if (q != hipSuccess) return fail(LST_E_DEVICE, hipGetErrorString(q));
  *done = 1;
  return LST_OK;
}

lst_status lst_event_wait(lst_event e) {
  if (!e) return fail(LST_E_INVALID, "lst_event_wait: NULL event");
  if (!e->synced) {
    if (e->status == LST_E_DEVICE) return fail(LST_E_DEVICE, "event failed at enqueue");
    HIP_TRY(hipEventSynchronize(e->done));
    e->synced = true;
    e->status = map_status(e->h_ctr[lst::C_STATUS]);
  }
  if (e->status != LST_OK) map_status(e->h_ctr[lst::C_STATUS]);
  return e->status;
}

lst_status lst_build_event(lst_geometry g, const lst_event_desc *ev, const lst_capacity *cap, void *workspace,
                           size_t ws_bytes, void *stream, lst_event *out) {
  lst_status s = lst_enqueue_event(g, ev, cap, workspace, ws_bytes, stream, out);
  if (s != LST_OK) return s;
  return lst_event_wait(*out);
}

lst_status lst_get_stage_counts(lst_event e, int64_t *counts, int64_t *required) {
  if (!e) return fail(LST_E_INVALID, "lst_get_stage_counts: NULL event");
  if (!e->synced) return fail(LST_E_STATE, "event not complete");
  const int *c = e->h_ctr;
  const int built[8] = {c[lst::C_NMD], c[lst::C_NLS], c[lst::C_NT3], c[lst::C_NT5],
                        e->ws.n_seeds, c[lst::C_NPT3], c[lst::C_NPT5], c[lst::C_NTC]};
  const int req[8] = {c[lst::C_RMD], c[lst::C_RLS], c[lst::C_RT3], c[lst::C_RT5],
                      e->ws.n_seeds, c[lst::C_RPT3], c[lst::C_RPT5], c[lst::C_NTC]};
  for (int i = 0; i < 8; ++i) {
    if (counts) counts[i] = built[i];
    if (required) required[i] = req[i];
  }
  return LST_OK;
}

lst_status lst_get_track_candidates(lst_event e, int32_t *n_tc, int32_t *n_hits_total, int32_t *type,
                                    int32_t *offsets, int32_t *hits) {
  if (!e || !n_tc || !n_hits_total) return fail(LST_E_INVALID, "lst_get_track_candidates: NULL argument");
  if (!e->synced) return fail(LST_E_STATE, "event not complete");
  if (e->status != LST_OK) return fail(LST_E_STATE, "event did not build (status " + std::to_string(e->status) + ")");
  const int n = e->h_ctr[lst::C_NTC], nh = e->h_ctr[lst::C_NTCHITS];
  *n_tc = n;
  *n_hits_total = nh;
  if (type && n > 0) HIP_TRY(hipMemcpy(type, e->ws.tc_type, sizeof(int) * n, hipMemcpyDeviceToHost));
  if (offsets) HIP_TRY(hipMemcpy(offsets, e->ws.tc_off, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
  if (hits && nh > 0) HIP_TRY(hipMemcpy(hits, e->ws.tc_hits, sizeof(int) * nh, hipMemcpyDeviceToHost));
  return LST_OK;
}

lst_status lst_get_stage_objects(lst_event e, int32_t stage, int32_t *n_out, int32_t *tuples, int32_t *flags,
                                 float *attrs) {
  if (!e || !n_out || stage < 0 || stage > 6) return fail(LST_E_INVALID, "lst_get_stage_objects: bad argument");
  if (!e->synced) return fail(LST_E_STATE, "event not complete");
  const int *c = e->h_ctr;
  const lst::Ws &w = e->ws;
  const int cnt[7] = {c[lst::C_NMD], c[lst::C_NLS], c[lst::C_NT3], c[lst::C_NT5], w.n_seeds, c[lst::C_NPT3],
                      c[lst::C_NPT5]};
  const int n = cnt[stage];
  *n_out = n;
  if (!tuples && !flags && !attrs) return LST_OK;
  // the MD table is needed to turn MD indices into hit indices
  std::vector<int2> mdh;
  HIP_TRY(d2h(mdh, w.md_hits, (size_t)c[lst::C_NMD]));
  auto put_md = [&](int32_t *dst, int md) { dst[0] = mdh[md].x; dst[1] = mdh[md].y; };
  std::vector<int> f(n > 0 ? n : 1, 1);
  std::vector<float> a((size_t)(n > 0 ? n : 1) * (kAttrW[stage] ? kAttrW[stage] : 1));
  std::vector<int> mds;  // n x k MD indices
  int k = 0;
  std::vector<int> seeds;
  if (stage == 0) {
    k = 1;
    mds.resize(n);
    for (int i = 0; i < n; ++i) mds[i] = i;
  } else if (stage == 1) {
    std::vector<int2> v; std::vector<float2> b;
    HIP_TRY(d2h(v, w.ls_md, n)); HIP_TRY(d2h(b, w.ls_beta, n));
    k = 2; mds.resize(2 * (size_t)n);
    for (int i = 0; i < n; ++i) { mds[2 * i] = v[i].x; mds[2 * i + 1] = v[i].y; a[2 * i] = b[i].x; a[2 * i + 1] = b[i].y; }
  } else if (stage == 2) {
    std::vector<int4> v; std::vector<float4> b;
    HIP_TRY(d2h(v, w.t3_md, n)); HIP_TRY(d2h(b, w.t3_attr, n));
    k = 3; mds.resize(3 * (size_t)n);
    for (int i = 0; i < n; ++i) {
      mds[3 * i] = v[i].x; mds[3 * i + 1] = v[i].y; mds[3 * i + 2] = v[i].z;
      a[4 * i] = b[i].x; a[4 * i + 1] = b[i].y; a[4 * i + 2] = b[i].z; a[4 * i + 3] = b[i].w;
    }
  } else if (stage == 3) {
    k = 5;
    HIP_TRY(d2h(mds, w.t5_md, 5 * (size_t)n));
    HIP_TRY(d2h(a, w.t5_attr, 8 * (size_t)n));
    HIP_TRY(d2h(f, w.t5_keep, n));
  } else if (stage == 4) {
    std::vector<float> p;
    HIP_TRY(d2h(p, w.pls, 8 * (size_t)n));
    HIP_TRY(d2h(f, w.pls_keep, n));
    for (int i = 0; i < n; ++i)
      for (int q = 0; q < 5; ++q) a[5 * i + q] = p[8 * i + q];
    seeds.resize(n);
    for (int i = 0; i < n; ++i) seeds[i] = i;
  } else {
    const bool five = stage == 6;
    std::vector<int2> so; std::vector<float4> b;
    HIP_TRY(d2h(so, five ? (const void *)w.pt5_so : (const void *)w.pt3_so, n));
    HIP_TRY(d2h(b, five ? (const void *)w.pt5_attr : (const void *)w.pt3_attr, n));
    HIP_TRY(d2h(f, five ? w.pt5_keep : w.pt3_keep, n));
    k = five ? 5 : 3;
    mds.resize((size_t)k * n);
    seeds.resize(n);
    if (five) {
      std::vector<int> t5md;
      HIP_TRY(d2h(t5md, w.t5_md, 5 * (size_t)c[lst::C_NT5]));
      for (int i = 0; i < n; ++i)
        for (int q = 0; q < 5; ++q) mds[5 * i + q] = t5md[5 * (size_t)so[i].y + q];
    } else {
      std::vector<int4> t3md;
      HIP_TRY(d2h(t3md, w.t3_md, (size_t)c[lst::C_NT3]));
      for (int i = 0; i < n; ++i) {
        mds[3 * i] = t3md[so[i].y].x; mds[3 * i + 1] = t3md[so[i].y].y; mds[3 * i + 2] = t3md[so[i].y].z;
      }
    }
    for (int i = 0; i < n; ++i) {
      seeds[i] = so[i].x;
      a[3 * i] = b[i].x; a[3 * i + 1] = b[i].y; a[3 * i + 2] = b[i].z;
    }
  }
  const int tw = kTupleW[stage];
  for (int i = 0; i < n; ++i) {
    int32_t *dst = tuples ? tuples + (size_t)i * tw : nullptr;
    if (!dst) continue;
    int o = 0;
    if (stage >= 4) dst[o++] = seeds[i];
    for (int q = 0; q < k; ++q, o += 2) put_md(dst + o, mds[(size_t)k * i + q]);
  }
  if (flags && n > 0) std::memcpy(flags, f.data(), sizeof(int) * n);
  if (attrs && kAttrW[stage] && n > 0) std::memcpy(attrs, a.data(), sizeof(float) * (size_t)n * kAttrW[stage]);
  return LST_OK;
}

int32_t lst_kernel_site_count(void) { return lst::kNumSites; }

const char *lst_kernel_site_name(int32_t site) {
  return (site >= 0 && site < lst::kNumSites) ? lst::kSiteNames[site] : nullptr;
}

lst_status lst_set_timed_site(int32_t site) {
  if (site < -1 || site >= lst::kNumSites) return fail(LST_E_INVALID, "lst_set_timed_site: no such launch site");
  g_timed_site.store(site);
  return LST_OK;
}

lst_status lst_get_site_time(lst_event e, float *ms) {
  if (!e || !ms) return fail(LST_E_INVALID, "lst_get_site_time: NULL argument");
  if (!e->synced) return fail(LST_E_STATE, "event not complete");
  if (e->timed_site < 0) return fail(LST_E_STATE, "no launch site was timed for this event");
  HIP_TRY(hipEventElapsedTime(ms, e->tbeg, e->tend));
  return LST_OK;
}

lst_status lst_release_event(lst_event e) {
  if (!e) return LST_OK;
  if (e->tbeg) drop(hipEventDestroy(e->tbeg));
  if (e->tend) drop(hipEventDestroy(e->tend));
  if (!e->synced && e->done) drop(hipEventSynchronize(e->done));
  if (e->done) drop(hipEventDestroy(e->done));
  if (e->h_ctr) drop(hipHostFree(e->h_ctr));
  delete e;
  return LST_OK;
}

}  // extern "C"
