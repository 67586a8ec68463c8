// C ABI of the LST library (include/lst.h): argument checks, geometry upload,
// workspace carving, enqueue of the kernel chain, result copies.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <unordered_map>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lst.h"
#include "lst_ws.hpp"

namespace {

// Last error message of the calling thread, in a fixed buffer (setting it
// allocates nothing, which the allocation-free entry point relies on).
thread_local char g_err[512];

lst_status fail(lst_status s, const char *msg) {
  snprintf(g_err, sizeof(g_err), "%s", msg);
  return s;
}
lst_status fail(lst_status s, const std::string &msg) { return fail(s, msg.c_str()); }

#define HIP_TRY(expr)                                                                               \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
    if (e_ != hipSuccess) return fail(LST_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kAlign = 256;
constexpr int kTupleW[7] = {2, 4, 6, 10, 1, 7, 11};
constexpr int kAttrW[7] = {0, 2, 4, 8, 5, 3, 3};
constexpr int64_t kMaxCap = 8000000;  // bounded by the two-level device scan (4096 x 2048)
constexpr int64_t kMaxTc = 4096L * 2048 - 1;  // pT5 + pT3 + T5 + pLS capacities: one scan of candidates
std::atomic<int> g_timed_site{-1};

}  // namespace

struct lst_geometry_s {
  lst::DevGeom g;
  int *d_off = nullptr, *d_tgt = nullptr, *d_info = nullptr;
  float4 *d_win = nullptr;
  float2 *d_t5cut = nullptr;  // per quintuplet category: chi2_xy, chi2_rz bounds
  int site_block[lst::kMaxSites] = {};  // launch shape of each tunable site (0 = default)
  float *d_pos = nullptr;  // per module: pos_lo, pos_up, lmin, lmax (kept to recompute the windows)
};

// Transverse impact-parameter bound of the selections unless set otherwise [cm].
constexpr double kD0MaxDefault = 0.1;

namespace {
// Quintuplet chi2 cuts per category (Section 2.3: set empirically for each
// category of quintuplets).  Category = the ordered kinds of the five anchor
// modules, innermost first, kind 0 barrel PS, 1 barrel 2S, 2 endcap PS,
// 3 endcap 2S; index sum_i kind_i 4^i.  The values are the 99.5% quantile of
// the circle-fit and r-z chi2 of quintuplets whose ten hits come from one
// generated track, on 20 calibration events (PU200-like, generator events
// 900-919, disjoint from the test and benchmark events), rounded up to three
// significant digits; categories with fewer than 50 such quintuplets take the
// quantile pooled over all categories.
constexpr double kT5Pooled[2] = {2.25, 2.7};
constexpr struct { int cat; double xy, rz; } kT5Cuts[] = {
    {320, 2.5, 2.83},    {336, 2.53, 2.5},    {672, 0.194, 2.55},  {680, 0.148, 2.58},  {682, 0.137, 2.77},
    {832, 2.06, 2.87},   {848, 2.01, 2.49},   {896, 0.342, 2.74},  {928, 0.3, 2.76},    {936, 0.278, 2.7},
    {938, 0.275, 2.91},  {960, 0.622, 2.88},  {976, 0.906, 2.45},  {992, 0.451, 2.87},  {1000, 0.392, 2.62},
    {1002, 0.408, 2.8},  {1008, 0.716, 2.5},  {1012, 1.19, 2.67},  {1016, 0.493, 2.52}, {1018, 0.492, 2.57},
    {1020, 0.729, 2.68}, {1022, 0.614, 2.64}, {1023, 0.928, 1.75},
};
// The calibrated table as float pairs (each value rounded once from double).
void t5_default_cuts(float2 *out) {
  for (int c = 0; c < 1024; ++c) out[c] = make_float2((float)kT5Pooled[0], (float)kT5Pooled[1]);
  for (const auto &e : kT5Cuts) out[e.cat] = make_float2((float)e.xy, (float)e.rz);
}
}  // namespace

// Events enqueued together share one batch: one descriptor array and one
// counter block in the workspace header, one completion event, one pinned
// read-back buffer.
struct lst_server_s;

struct lst_batch_s {
  lst_geometry geom = nullptr;
  int B = 0;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  lst::Ws *h_ws = nullptr;  // pinned: the descriptors uploaded to the header
  int *h_ctr = nullptr;     // pinned: copy of the B x C_COUNT counters
  std::atomic<int> refs{0};
  std::atomic<bool> synced{false};
  lst_server_s *server = nullptr;  // a server batch returns its workspace block here when freed
  size_t block_off = 0;
  bool failed = false;      // a HIP call failed at enqueue
  int timed_site = -1;      // launch site bracketed by tbeg/tend, or -1
  hipEvent_t tbeg = nullptr, tend = nullptr;
  lst_batch_s **owner = nullptr;  // a plan's pointer to its latest run, cleared when this batch is freed
  int device = 0;                 // device current when the batch was made (its events belong to it)
};

struct lst_event_s {
  lst_batch_s *batch = nullptr;
  int index = 0;
  const lst::Ws &ws() const { return batch->h_ws[index]; }
  const int *ctr() const { return batch->h_ctr + (size_t)index * lst::C_COUNT; }
  bool synced() const { return batch->synced; }
};

namespace lst {

size_t workspace_layout(int n_mod, int n_hits, int n_seeds, const Caps &c, Ws *w, char *base, int *ctr,
                        int n_hits_alloc, int n_seeds_alloc) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char * {
    off = (off + kAlign - 1) / kAlign * kAlign;
    char *p = base ? base + off : nullptr;
    off += bytes ? bytes : 1;
    return p;
  };
  const long N = n_hits_alloc >= 0 ? n_hits_alloc : n_hits, S = n_seeds_alloc >= 0 ? n_seeds_alloc : n_seeds;
  const long M = n_mod;
  const long md = c.md, ls = c.ls, t3 = c.t3, t5 = c.t5, p3 = c.pt3, p5 = c.pt5;
  const long tc = p5 + p3 + t5 + S;
#define I(n) reinterpret_cast<int *>(take(sizeof(int) * (size_t)(n)))
#define F(n) reinterpret_cast<float *>(take(sizeof(float) * (size_t)(n)))
#define I2(n) reinterpret_cast<int2 *>(take(sizeof(int2) * (size_t)(n)))
#define I4(n) reinterpret_cast<int4 *>(take(sizeof(int4) * (size_t)(n)))
#define F2(n) reinterpret_cast<float2 *>(take(sizeof(float2) * (size_t)(n)))
#define F4(n) reinterpret_cast<float4 *>(take(sizeof(float4) * (size_t)(n)))
  Ws t{};
  t.ctr = ctr;
  const long tiles = (long)n_coarse((int)M) * n_hit_tiles(N);
  t.boff = I(2 * M + 1); t.tile_hist = I(tiles + 1); t.tile_off = I(tiles + 1);
  t.hcp = F4(N + 1); t.hidx = I(N + 1); t.hpos = F4(N + 1);
  t.md_cnt = I(M + 1); t.md_off = I(M + 1); t.md_cache = I(kMdCache * M); t.md_part = I((long)kMdParts * M);
  t.md_bcache = I((long)kMdParts * kMdQCache * M); t.md_dense = I(M + 1);
  t.md_hits = I2(md); t.md_mod = I(md); t.md_pos = F4(md); t.md_stub = F2(md); t.mod_disc = F4(M);
  t.ls_cnt = I(md + 1); t.ls_off = I(md + 1); t.ls_md = I2(ls); t.ls_beta = F2(ls); t.ls_opos = F4(ls); t.ls_oinf = I(ls);
  t.ls_cache = I(kLsCache * md);
  t.ls_ovf_flag = I(md + 1); t.ls_ovf_off = I(md + 1); t.ls_ovf = I(md);
  t.t3_cnt = I(ls + 1); t.t3_off = I(ls + 1); t.t3_md = I4(t3); t.t3_attr = F4(t3); t.t3_first = F2(t3);
  t.t3_cache = I(kT3Cache * ls); t.t5_cache = I(kT5Cache * t3);
  t.t5_cnt = I(t3 + 1); t.t5_off = I(t3 + 1); t.t5_t3 = I2(t5); t.t5_md = I(5 * t5); t.t5_attr = F(8 * t5);
  t.t5_keep = I(t5); t.t5_first = F2(t5);
  t.inc_cnt = I(md + 1); t.inc_off = I(md + 1); t.inc_cur = I(md + 1); t.inc_list = I2(5 * t5);
  t.pls = F(8 * S); t.pls_keep = I(S); t.seed_order = I(S + 1);
  t.ph_cnt = I(N + 1); t.ph_off = I(N + 1); t.ph_cur = I(N + 1); t.ph_list = I(4 * S);
  t.pt3_cnt = I(S + 1); t.pt3_off = I(S + 1); t.pt5_cnt = I(S + 1); t.pt5_off = I(S + 1);
  t.pt3_cache = I(kPt3Cache * S); t.pt5_cache = I(kPt5Cache * S);
  t.pt3_cattr = F4(kPt3Cache * S); t.pt5_cattr = F4(kPt5Cache * S);
  t.pt3_so = I2(p3); t.pt5_so = I2(p5); t.pt3_attr = F4(p3); t.pt5_attr = F4(p5);
  t.pt3_keep = I(p3); t.pt5_keep = I(p5);
  t.o3_best = reinterpret_cast<unsigned long long *>(take(8 * (size_t)(t3 + 1)));
  t.o5_best = reinterpret_cast<unsigned long long *>(take(8 * (size_t)(t5 + 1)));
  const long nbins = kSeedBins;
  t.b3_cnt = I(nbins + 1); t.b3_off = I(nbins + 1); t.b3_cur = I(nbins + 1); t.b3_list = I(t3);
  t.b5_cnt = I(nbins + 1); t.b5_off = I(nbins + 1); t.b5_cur = I(nbins + 1); t.b5_list = I(t5);
  t.b3_pos = F4(t3); t.b5_pos = F4(t5);
  t.seed_used = I(S + 1); t.t5_used = I(t5 + 1);
  t.f_pt5 = I(p5 + 1); t.f_pt3 = I(p3 + 1); t.f_t5 = I(t5 + 1); t.f_pls = I(S + 1);
  t.p_pt5 = I(p5 + 1); t.p_pt3 = I(p3 + 1); t.p_t5 = I(t5 + 1); t.p_pls = I(S + 1);
  t.dir_pt5 = F4(p5); t.dir_pt3 = F4(p3); t.dir_t5 = F4(t5);
  t.bdir_pt5 = F4(p5); t.bdir_pt3 = F4(p3); t.bdir_t5 = F4(t5);
  t.boff_pt5 = I(129); t.boff_pt3 = I(129); t.boff_t5 = I(129);
  t.tc_type = I(tc); t.tc_off = I(tc + 1); t.tc_hits = I(14 * tc);
  t.tc_md = I(5 * tc); t.tc_kap = F2(tc);
  t.ext_n = I(tc); t.ext_t3 = I(tc); t.ext_cnt = I(tc + 1); t.ext_off = I(tc + 1); t.ext_hits = I(18 * tc);
  t.ext_attr = F4(tc);
  t.scan_tmp = I(4096);
#undef I
#undef F
#undef I2
#undef I4
#undef F2
#undef F4
  t.cap_md = (int)md; t.cap_ls = (int)ls; t.cap_t3 = (int)t3; t.cap_t5 = (int)t5;
  t.cap_pt3 = (int)p3; t.cap_pt5 = (int)p5;
  t.n_hits = n_hits; t.n_seeds = n_seeds;
  t.cap_tc = (int)(p5 + p3 + t5 + n_seeds);
  if (w && base) {
    const long N = n_hits, S = n_seeds;  // the jobs follow the event's own sizes
    int *ct = t.ctr;
    auto sj = [&](int id, const int *in, int *out, const int *n_dev, long n_fix, long n_cap, int *req, int *clamped,
                  long cap) { t.scans[id] = ScanJob{in, out, n_dev, (int)n_fix, (int)n_cap, req, clamped, (int)cap}; };
    const long nt = (long)n_coarse((int)M) * n_hit_tiles(n_hits);
    const long nt_cap = (long)n_coarse((int)M) * n_hit_tiles(n_hits_alloc >= 0 ? n_hits_alloc : n_hits);
    sj(SC_HITS, t.tile_hist, t.tile_off, nullptr, nt, nt_cap, ct + C_NOUTER, nullptr, 0);
    sj(SC_MD, t.md_cnt, t.md_off, nullptr, M, M, ct + C_RMD, ct + C_NMD, md);
    sj(SC_LS, t.ls_cnt, t.ls_off, ct + C_NMD, 0, md, ct + C_RLS, ct + C_NLS, ls);
    sj(SC_T3, t.t3_cnt, t.t3_off, ct + C_NLS, 0, ls, ct + C_RT3, ct + C_NT3, t3);
    sj(SC_T5, t.t5_cnt, t.t5_off, ct + C_NT3, 0, t3, ct + C_RT5, ct + C_NT5, t5);
    sj(SC_INC, t.inc_cnt, t.inc_off, ct + C_NMD, 0, md, ct + C_NINC, nullptr, 0);
    sj(SC_PH, t.ph_cnt, t.ph_off, nullptr, N, N, ct + C_NPH, nullptr, 0);
    sj(SC_PT3, t.pt3_cnt, t.pt3_off, nullptr, S, S, ct + C_RPT3, ct + C_NPT3, p3);
    sj(SC_PT5, t.pt5_cnt, t.pt5_off, nullptr, S, S, ct + C_RPT5, ct + C_NPT5, p5);
    sj(SC_F5, t.f_pt5, t.p_pt5, ct + C_NPT5, 0, p5, ct + C_NTC0, nullptr, 0);
    sj(SC_F3, t.f_pt3, t.p_pt3, ct + C_NPT3, 0, p3, ct + C_NTC1, nullptr, 0);
    sj(SC_FT5, t.f_t5, t.p_t5, ct + C_NT5, 0, t5, ct + C_NTC2, nullptr, 0);
    sj(SC_FPLS, t.f_pls, t.p_pls, nullptr, S, S, ct + C_NTC3, nullptr, 0);
    sj(SC_B3, t.b3_cnt, t.b3_off, nullptr, nbins, nbins, ct + C_NB3, nullptr, 0);
    sj(SC_B5, t.b5_cnt, t.b5_off, nullptr, nbins, nbins, ct + C_NB5, nullptr, 0);
    sj(SC_LSOVF, t.ls_ovf_flag, t.ls_ovf_off, ct + C_NMD, 0, md, ct + C_NLSOVF, nullptr, 0);
    sj(SC_EXT, t.ext_cnt, t.ext_off, ct + C_NTC, 0, p5 + p3 + t5 + S, ct + C_NEXTHITS, nullptr, 0);
    // arrays indexed by MDs, triplets or quintuplets are cleared up to the built count
    // (the clears run after it is known), not the capacity
    auto fj = [&](int id, int *p, long n, const int *n_dev = nullptr, int mul = 1) {
      t.fills[id] = FillJob{p, n, n_dev, mul};
    };
    fj(FL_CTR, ct, C_COUNT);
    fj(FL_INC_CNT, t.inc_cnt, md + 1, ct + C_NMD);
    fj(FL_INC_CUR, t.inc_cur, md + 1, ct + C_NMD);
    fj(FL_PH_CNT, t.ph_cnt, N + 1);
    fj(FL_PH_CUR, t.ph_cur, N + 1);
    fj(FL_O3_BEST, reinterpret_cast<int *>(t.o3_best), 2 * (t3 + 1), ct + C_NT3, 2);
    fj(FL_O5_BEST, reinterpret_cast<int *>(t.o5_best), 2 * (t5 + 1), ct + C_NT5, 2);
    fj(FL_SEED_USED, t.seed_used, S + 1);
    fj(FL_T5_USED, t.t5_used, t5 + 1, ct + C_NT5);
    fj(FL_B3_CNT, t.b3_cnt, nbins + 1);
    fj(FL_B3_CUR, t.b3_cur, nbins + 1);
    fj(FL_B5_CNT, t.b5_cnt, nbins + 1);
    fj(FL_B5_CUR, t.b5_cur, nbins + 1);
  }
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

const char *lst_last_error(void) { return g_err; }

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
  // track candidates (pT5 + pT3 + T5 + pLS) go through one device scan: keep their sum in it
  const int64_t room = kMaxTc - S;
  const int64_t sum = out->pt5 + out->pt3 + out->t5;
  if (sum > room) {
    out->t5 = std::max<int64_t>(1, out->t5 * room / sum);
    out->pt3 = std::max<int64_t>(1, out->pt3 * room / sum);
    out->pt5 = std::max<int64_t>(1, out->pt5 * room / sum);
  }
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
    if (d->map_offsets[m + 1] - d->map_offsets[m] > 128)
      return fail(LST_E_INVALID, "more than 128 module-map targets for one module");
  if (M > lst::kMaxModules) return fail(LST_E_INVALID, "more than 32,768 modules (the hit bucketing's limit)");
  auto *g = new (std::nothrow) lst_geometry_s();
  if (!g) return fail(LST_E_NOMEM, "host allocation failed");
  std::vector<int> info(M);
  for (int m = 0; m < M; ++m) info[m] = (d->type[m] & 1) | ((d->subdet[m] & 1) << 1);  // 2 bits (packed with MD indices)
  auto cleanup = [&]() {
    drop(hipFree(g->d_off)); drop(hipFree(g->d_tgt)); drop(hipFree(g->d_info)); drop(hipFree(g->d_win));
    drop(hipFree(g->d_pos)); drop(hipFree(g->d_t5cut));
    delete g;
  };
  float *&d_pos = g->d_pos;
  if (hipMalloc(&g->d_off, sizeof(int) * (M + 1)) != hipSuccess ||
      hipMalloc(&g->d_tgt, sizeof(int) * (E > 0 ? E : 1)) != hipSuccess ||
      hipMalloc(&g->d_info, sizeof(int) * M) != hipSuccess || hipMalloc(&g->d_win, sizeof(float4) * M) != hipSuccess ||
      hipMalloc(&d_pos, sizeof(float) * 4 * M) != hipSuccess || hipMalloc(&g->d_t5cut, sizeof(float2) * 1024) != hipSuccess) {
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
    std::vector<float2> cuts(1024);
    t5_default_cuts(cuts.data());
    e = hipMemcpy(g->d_t5cut, cuts.data(), sizeof(float2) * 1024, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) {
    lst::launch_module_windows(g->d_info, d_pos, d_pos + M, d_pos + 2 * M, d_pos + 3 * M, M, kD0MaxDefault, g->d_win,
                               nullptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    cleanup();
    return fail(LST_E_DEVICE, std::string("lst_load_geometry: ") + hipGetErrorString(e));
  }
  g->g.n_mod = M;
  g->g.n_edges = E;
  g->g.map_off = g->d_off;
  g->g.map_tgt = g->d_tgt;
  g->g.win = g->d_win;
  g->g.info = g->d_info;
  g->g.ext = 0;
  g->g.d0max = (float)kD0MaxDefault;
  g->g.stub16 = 0;
  g->g.t5cut = g->d_t5cut;
  g->g.tiles = lst::kTilesDefault;
  *out = g;
  return LST_OK;
}

lst_status lst_set_t5_cuts(lst_geometry g, const float *xy, const float *rz) {
  if (!g) return fail(LST_E_INVALID, "lst_set_t5_cuts: NULL geometry");
  std::vector<float2> cuts(1024);
  t5_default_cuts(cuts.data());
  for (int c = 0; c < 1024; ++c) {
    if (xy) cuts[c].x = xy[c];
    if (rz) cuts[c].y = rz[c];
    if (std::isnan(cuts[c].x) || std::isnan(cuts[c].y)) return fail(LST_E_INVALID, "lst_set_t5_cuts: NaN cut");
  }
  HIP_TRY(hipMemcpy(g->d_t5cut, cuts.data(), sizeof(float2) * 1024, hipMemcpyHostToDevice));
  return LST_OK;
}

lst_status lst_get_default_t5_cuts(float *xy, float *rz) {
  if (!xy || !rz) return fail(LST_E_INVALID, "lst_get_default_t5_cuts: NULL argument");
  float2 cuts[1024];
  t5_default_cuts(cuts);
  for (int c = 0; c < 1024; ++c) { xy[c] = cuts[c].x; rz[c] = cuts[c].y; }
  return LST_OK;
}

lst_status lst_get_t5_cuts(lst_geometry g, float *xy, float *rz) {
  if (!g || !xy || !rz) return fail(LST_E_INVALID, "lst_get_t5_cuts: NULL argument");
  std::vector<float2> cuts(1024);
  HIP_TRY(hipMemcpy(cuts.data(), g->d_t5cut, sizeof(float2) * 1024, hipMemcpyDeviceToHost));
  for (int c = 0; c < 1024; ++c) { xy[c] = cuts[c].x; rz[c] = cuts[c].y; }
  return LST_OK;
}

lst_status lst_set_stub_precision(lst_geometry g, int32_t bits) {
  if (!g || (bits != 16 && bits != 32)) return fail(LST_E_INVALID, "lst_set_stub_precision: bits must be 16 or 32");
  g->g.stub16 = bits == 16 ? 1 : 0;
  return LST_OK;
}

lst_status lst_set_impact_bound(lst_geometry g, double d0_max) {
  if (!g || !(d0_max > 0.0) || !(d0_max <= 10.0))
    return fail(LST_E_INVALID, "lst_set_impact_bound: geometry NULL or bound outside (0, 10] cm");
  const int M = g->g.n_mod;
  float *p = g->d_pos;
  lst::launch_module_windows(g->d_info, p, p + M, p + 2 * M, p + 3 * M, M, d0_max, g->d_win, nullptr);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipDeviceSynchronize());
  g->g.d0max = (float)d0_max;
  return LST_OK;
}

lst_status lst_set_track_extensions(lst_geometry g, int32_t enable) {
  if (!g || (enable != 0 && enable != 1)) return fail(LST_E_INVALID, "lst_set_track_extensions: bad argument");
  g->g.ext = enable;
  return LST_OK;
}

lst_status lst_release_geometry(lst_geometry g) {
  if (!g) return LST_OK;
  drop(hipFree(g->d_off)); drop(hipFree(g->d_tgt)); drop(hipFree(g->d_info)); drop(hipFree(g->d_win));
  drop(hipFree(g->d_pos)); drop(hipFree(g->d_t5cut));
  delete g;
  return LST_OK;
}

lst_status lst_get_module_constants(lst_geometry g, float *out) {
  if (!g || !out) return fail(LST_E_INVALID, "lst_get_module_constants: NULL argument");
  HIP_TRY(hipMemcpy(out, g->d_win, sizeof(float4) * g->g.n_mod, hipMemcpyDeviceToHost));
  return LST_OK;
}

// ---------------------------------------------------------------- batches
// Workspace of a batch of B events: header (B descriptors, B x C_COUNT
// counters), then one region per event.
static size_t header_bytes(int B) {
  const size_t d = ((sizeof(lst::Ws) * (size_t)B + kAlign - 1) / kAlign) * kAlign;
  const size_t c = ((sizeof(int) * lst::C_COUNT * (size_t)B + kAlign - 1) / kAlign) * kAlign;
  return d + c;
}

static lst_status resolve_caps(int B, const int32_t *nh, const int32_t *ns, const lst_capacity *cap,
                               std::vector<lst::Caps> &out) {
  out.resize(B);
  for (int i = 0; i < B; ++i) {
    if (nh[i] < 0 || ns[i] < 0 || nh[i] > kMaxCap || ns[i] > kMaxCap / 4)
      return fail(LST_E_INVALID, "n_hits above 8e6 or n_seeds above 2e6, or negative");
    lst_capacity c;
    if (cap) c = cap[i]; else lst_default_capacity(nh[i], ns[i], &c);
    lst_status s = check_caps(c);
    if (s != LST_OK) return s;
    if (c.pt5 + c.pt3 + c.t5 + ns[i] > kMaxTc)
      return fail(LST_E_INVALID, "capacities pT5 + pT3 + T5 + seeds above 8,388,607 (one device scan)");
    out[i] = lst::Caps{c.md, c.ls, c.t3, c.t5, c.pt3, c.pt5};
  }
  return LST_OK;
}

static size_t batch_bytes(int n_mod, int B, const int32_t *nh, const int32_t *ns, const std::vector<lst::Caps> &c) {
  size_t off = header_bytes(B);
  for (int i = 0; i < B; ++i) off += lst::workspace_layout(n_mod, nh[i], ns[i], c[i], nullptr, nullptr, nullptr);
  return off;
}

// Pinned host buffers and HIP events of freed batches, kept for the next batch
// (allocating pinned memory costs far more than a batch's other host work).
// Buffers are kept by power-of-two size class, events per device; at most
// kPoolPinnedMax bytes of buffers are kept, the rest is freed.  Nothing is
// released at process exit.
constexpr int kPoolClasses = 24;               // size classes 2^0 .. 2^23 bytes
constexpr size_t kPoolPinnedMax = 64u << 20;
struct HostPool {
  std::mutex mu;
  std::vector<void *> pinned[kPoolClasses];
  size_t pinned_bytes = 0;
  std::unordered_map<int, std::vector<hipEvent_t>> sync_events, timing_events;
};
static HostPool &host_pool() {
  static HostPool *p = new HostPool();  // never destroyed: no HIP calls during static teardown
  return *p;
}
static int size_class(size_t n) {
  int k = 0;
  while (((size_t)1 << k) < n) ++k;
  return k;
}
static void *pinned_get(size_t n) {
  const int k = size_class(n);
  if (k < kPoolClasses) {
    HostPool &P = host_pool();
    std::lock_guard<std::mutex> lk(P.mu);
    if (!P.pinned[k].empty()) {
      void *q = P.pinned[k].back();
      P.pinned[k].pop_back();
      P.pinned_bytes -= (size_t)1 << k;
      return q;
    }
  }
  void *q = nullptr;
  if (hipHostMalloc(&q, k < kPoolClasses ? (size_t)1 << k : n, hipHostMallocDefault) != hipSuccess) return nullptr;
  return q;
}
static void pinned_put(void *q, size_t n) {
  if (!q) return;
  const int k = size_class(n);
  if (k < kPoolClasses) {
    HostPool &P = host_pool();
    std::lock_guard<std::mutex> lk(P.mu);
    if (P.pinned_bytes + ((size_t)1 << k) <= kPoolPinnedMax) {
      P.pinned[k].push_back(q);
      P.pinned_bytes += (size_t)1 << k;
      return;
    }
  }
  drop(hipHostFree(q));
}
static hipEvent_t event_get(int device, bool timing) {
  {
    HostPool &P = host_pool();
    std::lock_guard<std::mutex> lk(P.mu);
    auto &v = (timing ? P.timing_events : P.sync_events)[device];
    if (!v.empty()) {
      hipEvent_t e = v.back();
      v.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if ((timing ? hipEventCreate(&e) : hipEventCreateWithFlags(&e, hipEventDisableTiming)) != hipSuccess) return nullptr;
  return e;
}
static void event_put(int device, hipEvent_t e, bool timing) {
  if (!e) return;
  HostPool &P = host_pool();
  std::lock_guard<std::mutex> lk(P.mu);
  auto &v = (timing ? P.timing_events : P.sync_events)[device];
  if (v.size() < 4096) {
    v.push_back(e);
    return;
  }
  drop(hipEventDestroy(e));
}
// Pinned buffers and completion event of a new batch of B events (false on failure).
static bool batch_host_resources(lst_batch_s *b, int B) {
  if (hipGetDevice(&b->device) != hipSuccess) return false;
  b->h_ctr = static_cast<int *>(pinned_get(sizeof(int) * lst::C_COUNT * B));
  b->h_ws = static_cast<lst::Ws *>(pinned_get(sizeof(lst::Ws) * B));
  b->done = event_get(b->device, false);
  return b->h_ctr && b->h_ws && b->done;
}

static void server_release_batch(lst_server_s *s, lst_batch_s *b);

static void release_batch_ref(lst_batch_s *b) {
  if (--b->refs > 0) return;
  if (b->owner && *b->owner == b) *b->owner = nullptr;
  if (b->server) server_release_batch(b->server, b);
  if (!b->synced && b->done) drop(hipEventSynchronize(b->done));
  event_put(b->device, b->tbeg, true);
  event_put(b->device, b->tend, true);
  event_put(b->device, b->done, false);
  pinned_put(b->h_ctr, sizeof(int) * lst::C_COUNT * b->B);
  pinned_put(b->h_ws, sizeof(lst::Ws) * b->B);
  delete b;
}

static lst_status map_status(int st) {
  if (st & (lst::ST_BAD_HIT | lst::ST_BAD_SEED))
    return fail(LST_E_INVALID, (st & lst::ST_BAD_HIT) ? "invalid hit data (module/sensor out of range or non-finite)"
                                                      : "invalid seed data (hit index, charge or momentum)");
  if (st & lst::ST_CAPACITY) return fail(LST_E_CAPACITY, "object capacity exceeded; see lst_get_stage_counts");
  return LST_OK;
}

lst_status lst_batch_workspace_bytes(lst_geometry g, int32_t B, const int32_t *n_hits, const int32_t *n_seeds,
                                     const lst_capacity *cap, size_t *bytes) {
  if (!g || !bytes || B < 1 || B > 65535 || !n_hits || !n_seeds)
    return fail(LST_E_INVALID, "lst_batch_workspace_bytes: bad argument");
  std::vector<lst::Caps> c;
  lst_status s = resolve_caps(B, n_hits, n_seeds, cap, c);
  if (s != LST_OK) return s;
  *bytes = batch_bytes(g->g.n_mod, B, n_hits, n_seeds, c);
  return LST_OK;
}

lst_status lst_workspace_bytes(lst_geometry g, int32_t n_hits, int32_t n_seeds, const lst_capacity *cap,
                               size_t *bytes) {
  return lst_batch_workspace_bytes(g, 1, &n_hits, &n_seeds, cap, bytes);
}

// The hit bucketing scans one count per (coarse bucket, tile of input hits):
// an event must keep that within one device scan on this geometry.
static lst_status check_bucketing(lst_geometry g, int64_t n_hits) {
  const int64_t items = (int64_t)lst::n_coarse(g->g.n_mod) * lst::n_hit_tiles(n_hits);
  if (items > kMaxTc) {
    char msg[200];
    snprintf(msg, sizeof(msg), "%lld hits: above what the hit bucketing scans on a detector of %d modules",
             (long long)n_hits, g->g.n_mod);
    return fail(LST_E_INVALID, msg);
  }
  return LST_OK;
}

static lst_status check_event_desc(const lst_event_desc &ev) {
  if (ev.n_hits < 0 || ev.n_seeds < 0) return fail(LST_E_INVALID, "negative n_hits or n_seeds");
  if (ev.n_hits > kMaxCap || ev.n_seeds > kMaxCap)
    return fail(LST_E_INVALID, "more than 8,000,000 hits or seeds in one event (the device scans' limit)");
  if (ev.n_hits > 0 && (!ev.x || !ev.y || !ev.z || !ev.module || !ev.sensor))
    return fail(LST_E_INVALID, "hit arrays missing");
  if (ev.n_seeds > 0 && (!ev.px || !ev.py || !ev.pz || !ev.q || !ev.hits4))
    return fail(LST_E_INVALID, "seed arrays missing");
  if (ev.n_seeds > 0 && ev.n_hits == 0) return fail(LST_E_INVALID, "seeds without hits");
  return LST_OK;
}

// Lays out B events in the workspace at `base` (batch_bytes() bytes), uploads
// their descriptors and enqueues the chain and the counter read-back on
// `stream`.  The returned batch holds one reference per event.
static lst_status enqueue_batch_at(lst_geometry g, int B, const lst_event_desc *evs, const std::vector<lst::Caps> &caps,
                                   char *base, hipStream_t stream, lst_batch_s **out, int timed_site = -2) {
  *out = nullptr;
  auto *b = new (std::nothrow) lst_batch_s();
  if (!b) return fail(LST_E_NOMEM, "host allocation failed");
  b->geom = g;
  b->B = B;
  b->stream = stream;
  b->refs = B;
  if (!batch_host_resources(b, B)) {
    b->refs = 1;
    release_batch_ref(b);
    return fail(LST_E_DEVICE, "pinned buffers or event creation failed");
  }
  lst::Ws *d_ws = reinterpret_cast<lst::Ws *>(base);
  int *d_ctr = reinterpret_cast<int *>(base + ((sizeof(lst::Ws) * (size_t)B + kAlign - 1) / kAlign) * kAlign);
  size_t off = header_bytes(B);
  lst::Ws bound{};
  for (int i = 0; i < B; ++i) {
    lst::Ws &w = b->h_ws[i];
    const lst_event_desc &ev = evs[i];
    off += lst::workspace_layout(g->g.n_mod, ev.n_hits, ev.n_seeds, caps[i], &w, base + off,
                                 d_ctr + (size_t)i * lst::C_COUNT);
    w.x = ev.x; w.y = ev.y; w.z = ev.z; w.module = ev.module; w.sensor = ev.sensor;
    w.px = ev.px; w.py = ev.py; w.pz = ev.pz; w.q = ev.q; w.hits4 = ev.hits4;
    bound.n_hits = std::max(bound.n_hits, w.n_hits);
    bound.n_seeds = std::max(bound.n_seeds, w.n_seeds);
    bound.cap_md = std::max(bound.cap_md, w.cap_md);
    bound.cap_ls = std::max(bound.cap_ls, w.cap_ls);
    bound.cap_t3 = std::max(bound.cap_t3, w.cap_t3);
    bound.cap_t5 = std::max(bound.cap_t5, w.cap_t5);
    bound.cap_pt3 = std::max(bound.cap_pt3, w.cap_pt3);
    bound.cap_pt5 = std::max(bound.cap_pt5, w.cap_pt5);
    bound.cap_tc = std::max(bound.cap_tc, w.cap_tc);
  }
  lst::KernelTimer kt{-1, nullptr, nullptr};
  const int site = timed_site >= -1 ? timed_site : g_timed_site.load();
  if (site >= 0 && (b->tbeg = event_get(b->device, true)) && (b->tend = event_get(b->device, true))) {
    kt = lst::KernelTimer{site, b->tbeg, b->tend};
    b->timed_site = site;
  }
  hipError_t he = hipMemcpyAsync(d_ws, b->h_ws, sizeof(lst::Ws) * B, hipMemcpyHostToDevice, stream);
  if (he == hipSuccess) {
    lst::enqueue_chain(g->g, d_ws, B, bound, stream, b->timed_site >= 0 ? &kt : nullptr, g->site_block);
    he = hipGetLastError();
  }
  if (he == hipSuccess)
    he = hipMemcpyAsync(b->h_ctr, d_ctr, sizeof(int) * lst::C_COUNT * B, hipMemcpyDeviceToHost, stream);
  if (he == hipSuccess) he = hipEventRecord(b->done, stream);
  if (he != hipSuccess) b->failed = true;
  *out = b;
  if (he != hipSuccess) return fail(LST_E_DEVICE, std::string("enqueue: ") + hipGetErrorString(he));
  return LST_OK;
}

static lst_status make_events(lst_batch_s *b, int n, lst_event *out) {
  for (int i = 0; i < n; ++i) {
    auto *e = new (std::nothrow) lst_event_s();
    if (!e) {
      for (int k = i; k < n; ++k) release_batch_ref(b);
      return fail(LST_E_NOMEM, "host allocation failed");
    }
    e->batch = b;
    e->index = i;
    out[i] = e;
  }
  return LST_OK;
}

lst_status lst_enqueue_batch(lst_geometry g, int32_t B, const lst_event_desc *evs, const lst_capacity *cap,
                             void *workspace, size_t ws_bytes, void *stream, lst_event *out) {
  if (!out) return fail(LST_E_INVALID, "lst_enqueue_batch: NULL out");
  if (!g || !evs || !workspace || B < 1 || B > 65535) return fail(LST_E_INVALID, "lst_enqueue_batch: bad argument");
  for (int i = 0; i < B; ++i) out[i] = nullptr;
  std::vector<int32_t> nh(B), ns(B);
  for (int i = 0; i < B; ++i) {
    lst_status s = check_event_desc(evs[i]);
    if (s == LST_OK) s = check_bucketing(g, evs[i].n_hits);
    if (s != LST_OK) return s;
    nh[i] = evs[i].n_hits;
    ns[i] = evs[i].n_seeds;
  }
  std::vector<lst::Caps> caps;
  lst_status s = resolve_caps(B, nh.data(), ns.data(), cap, caps);
  if (s != LST_OK) return s;
  const size_t need = batch_bytes(g->g.n_mod, B, nh.data(), ns.data(), caps);
  if (ws_bytes < need) return fail(LST_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return fail(LST_E_INVALID, "workspace not 256-byte aligned");
  lst_batch_s *b = nullptr;
  lst_status es = enqueue_batch_at(g, B, evs, caps, reinterpret_cast<char *>(workspace),
                                   reinterpret_cast<hipStream_t>(stream), &b);
  if (!b) return es;
  std::string msg = g_err;  // make_events may overwrite it
  lst_status ms = make_events(b, B, out);
  if (ms != LST_OK) return ms;
  if (es != LST_OK) snprintf(g_err, sizeof(g_err), "%s", msg.c_str());
  return es;
}

lst_status lst_enqueue_event(lst_geometry g, const lst_event_desc *ev, const lst_capacity *cap, void *workspace,
                             size_t ws_bytes, void *stream, lst_event *out) {
  if (!out) return fail(LST_E_INVALID, "lst_enqueue_event: NULL out");
  *out = nullptr;
  if (!ev) return fail(LST_E_INVALID, "lst_enqueue_event: NULL event");
  return lst_enqueue_batch(g, 1, ev, cap, workspace, ws_bytes, stream, out);
}

lst_status lst_event_query(lst_event e, int32_t *done) {
  if (!e || !done) return fail(LST_E_INVALID, "lst_event_query: NULL argument");
  lst_batch_s *b = e->batch;
  if (b->synced) { *done = 1; return LST_OK; }
  if (b->failed) return fail(LST_E_DEVICE, "event failed at enqueue");
  hipError_t q = hipEventQuery(b->done);
  if (q == hipErrorNotReady) { *done = 0; return LST_OK; }
  if (q != hipSuccess) return fail(LST_E_DEVICE, hipGetErrorString(q));
  *done = 1;
  return LST_OK;
}

lst_status lst_event_wait(lst_event e) {
  if (!e) return fail(LST_E_INVALID, "lst_event_wait: NULL event");
  lst_batch_s *b = e->batch;
  if (b->failed) return fail(LST_E_DEVICE, "event failed at enqueue");
  if (!b->synced) {
    HIP_TRY(hipEventSynchronize(b->done));
    b->synced = true;
  }
  return map_status(e->ctr()[lst::C_STATUS]);
}

lst_status lst_build_event(lst_geometry g, const lst_event_desc *ev, const lst_capacity *cap, void *workspace,
                           size_t ws_bytes, void *stream, lst_event *out) {
  lst_status s = lst_enqueue_event(g, ev, cap, workspace, ws_bytes, stream, out);
  if (s != LST_OK) return s;
  return lst_event_wait(*out);
}

// ------------------------------------------------ allocation-free entry point
// The workspace of lst_build_event_static: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never uses its name as an
// address: the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};

// A failed HIP call, reported without allocating.
lst_status fail_hip(const char *what, hipError_t e) {
  snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
  return LST_E_DEVICE;
}

// Device address of `scratch` on the current device (looked up on the first call there).
lst_status scratch_ptr(char **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip("hipGetDevice", e);
  if (dev < 0 || dev >= kMaxDevices) return fail(LST_E_DEVICE, "lst_build_event_static: device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip("hipGetSymbolAddress(scratch)", e);
    if (!p) return fail(LST_E_DEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = static_cast<char *>(p);
  }
  *out = g_scratch_ptr[dev];
  return LST_OK;
}
}  // namespace

lst_status lst_static_workspace_bytes(size_t *bytes) {
  if (!bytes) return fail(LST_E_INVALID, "lst_static_workspace_bytes: NULL argument");
  *bytes = kScratchBytes;
  return LST_OK;
}

lst_status lst_build_event_static(lst_geometry g, const lst_event_desc *ev, const lst_capacity *cap, void *stream,
                                  int32_t max_tc, int32_t max_tc_hits, int32_t *type, int32_t *offsets,
                                  int32_t *hits, int32_t *counts) {
  if (!g || !ev || !counts || !offsets || max_tc < 0 || max_tc_hits < 0 || (max_tc > 0 && !type) ||
      (max_tc_hits > 0 && !hits))
    return fail(LST_E_INVALID, "lst_build_event_static: bad argument");
  lst_status s = check_event_desc(*ev);
  if (s == LST_OK) s = check_bucketing(g, ev->n_hits);
  if (s != LST_OK) return s;
  if (ev->n_seeds > kMaxCap / 4) return fail(LST_E_INVALID, "n_seeds above 2e6");
  lst_capacity c;
  if (cap) c = *cap; else lst_default_capacity(ev->n_hits, ev->n_seeds, &c);
  s = check_caps(c);
  if (s != LST_OK) return s;
  if (c.pt5 + c.pt3 + c.t5 + ev->n_seeds > kMaxTc)
    return fail(LST_E_INVALID, "capacities pT5 + pT3 + T5 + seeds above 8,388,607 (one device scan)");
  const lst::Caps caps{c.md, c.ls, c.t3, c.t5, c.pt3, c.pt5};
  const size_t head = header_bytes(1);
  const size_t need = head + lst::workspace_layout(g->g.n_mod, ev->n_hits, ev->n_seeds, caps, nullptr, nullptr, nullptr);
  if (need > kScratchBytes) {
    char msg[200];
    snprintf(msg, sizeof(msg), "lst_build_event_static: event needs %zu bytes, above the static workspace of %zu",
             need, kScratchBytes);
    return fail(LST_E_NOMEM, msg);
  }
  char *base = nullptr;
  s = scratch_ptr(&base);
  if (s != LST_OK) return s;
  lst::Ws *d_ws = reinterpret_cast<lst::Ws *>(base);
  int *d_ctr = reinterpret_cast<int *>(base + ((sizeof(lst::Ws) + kAlign - 1) / kAlign) * kAlign);
  lst::Ws w{};
  lst::workspace_layout(g->g.n_mod, ev->n_hits, ev->n_seeds, caps, &w, base + head, d_ctr);
  w.x = ev->x; w.y = ev->y; w.z = ev->z; w.module = ev->module; w.sensor = ev->sensor;
  w.px = ev->px; w.py = ev->py; w.pz = ev->pz; w.q = ev->q; w.hits4 = ev->hits4;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  lst::launch_put_desc(w, d_ws, st);
  lst::enqueue_chain(g->g, d_ws, 1, w, st, nullptr, g->site_block);
  lst::launch_tc_export(d_ws, max_tc, max_tc_hits, type, offsets, hits, counts, st);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail_hip("lst_build_event_static: launch", e);
  return LST_OK;
}

static lst_status event_ok(lst_event e) {
  if (!e->synced()) return fail(LST_E_STATE, "event not complete");
  return LST_OK;
}

lst_status lst_get_stage_counts(lst_event e, int64_t *counts, int64_t *required) {
  if (!e) return fail(LST_E_INVALID, "lst_get_stage_counts: NULL event");
  if (event_ok(e) != LST_OK) return LST_E_STATE;
  const int *c = e->ctr();
  const int ns = e->ws().n_seeds;
  const int built[8] = {c[lst::C_NMD], c[lst::C_NLS], c[lst::C_NT3], c[lst::C_NT5],
                        ns, c[lst::C_NPT3], c[lst::C_NPT5], c[lst::C_NTC]};
  const int req[8] = {c[lst::C_RMD], c[lst::C_RLS], c[lst::C_RT3], c[lst::C_RT5],
                      ns, c[lst::C_RPT3], c[lst::C_RPT5], c[lst::C_NTC]};
  for (int i = 0; i < 8; ++i) {
    if (counts) counts[i] = built[i];
    if (required) required[i] = req[i];
  }
  return LST_OK;
}

lst_status lst_get_track_candidates(lst_event e, int32_t *n_tc, int32_t *n_hits_total, int32_t *type,
                                    int32_t *offsets, int32_t *hits) {
  if (!e || !n_tc || !n_hits_total) return fail(LST_E_INVALID, "lst_get_track_candidates: NULL argument");
  if (event_ok(e) != LST_OK) return LST_E_STATE;
  const int st = e->ctr()[lst::C_STATUS];
  if (st != 0) return fail(LST_E_STATE, "event did not build (status flags " + std::to_string(st) + ")");
  const lst::Ws &w = e->ws();
  const int n = e->ctr()[lst::C_NTC], nh = e->ctr()[lst::C_NTCHITS];
  *n_tc = n;
  *n_hits_total = nh;
  if (type && n > 0) HIP_TRY(hipMemcpy(type, w.tc_type, sizeof(int) * n, hipMemcpyDeviceToHost));
  if (offsets) HIP_TRY(hipMemcpy(offsets, w.tc_off, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
  if (hits && nh > 0) HIP_TRY(hipMemcpy(hits, w.tc_hits, sizeof(int) * nh, hipMemcpyDeviceToHost));
  return LST_OK;
}

lst_status lst_get_extended_track_candidates(lst_event e, int32_t *n_tc, int32_t *n_hits_total, int32_t *type,
                                             int32_t *offsets, int32_t *hits, int32_t *n_added, int32_t *t3,
                                             float *attrs) {
  if (!e || !n_tc || !n_hits_total) return fail(LST_E_INVALID, "lst_get_extended_track_candidates: NULL argument");
  if (event_ok(e) != LST_OK) return LST_E_STATE;
  const int st = e->ctr()[lst::C_STATUS];
  if (st != 0) return fail(LST_E_STATE, "event did not build (status flags " + std::to_string(st) + ")");
  if (e->ctr()[lst::C_EXT] != 1)
    return fail(LST_E_STATE, "track extensions were not enabled on the geometry when the event was enqueued");
  const lst::Ws &w = e->ws();
  const int n = e->ctr()[lst::C_NTC], nh = e->ctr()[lst::C_NEXTHITS];
  *n_tc = n;
  *n_hits_total = nh;
  if (type && n > 0) HIP_TRY(hipMemcpy(type, w.tc_type, sizeof(int) * n, hipMemcpyDeviceToHost));
  if (offsets) HIP_TRY(hipMemcpy(offsets, w.ext_off, sizeof(int) * (n + 1), hipMemcpyDeviceToHost));
  if (hits && nh > 0) HIP_TRY(hipMemcpy(hits, w.ext_hits, sizeof(int) * nh, hipMemcpyDeviceToHost));
  if (n_added && n > 0) HIP_TRY(hipMemcpy(n_added, w.ext_n, sizeof(int) * n, hipMemcpyDeviceToHost));
  if (t3 && n > 0) HIP_TRY(hipMemcpy(t3, w.ext_t3, sizeof(int) * n, hipMemcpyDeviceToHost));
  if (attrs && n > 0) {
    std::vector<float4> a;
    HIP_TRY(d2h(a, w.ext_attr, (size_t)n));
    for (int i = 0; i < n; ++i) {
      attrs[3 * (size_t)i] = a[i].x;
      attrs[3 * (size_t)i + 1] = a[i].y;
      attrs[3 * (size_t)i + 2] = a[i].z;
    }
  }
  return LST_OK;
}

lst_status lst_get_stage_objects(lst_event e, int32_t stage, int32_t *n_out, int32_t *tuples, int32_t *flags,
                                 float *attrs) {
  if (!e || !n_out || stage < 0 || stage > 6) return fail(LST_E_INVALID, "lst_get_stage_objects: bad argument");
  if (event_ok(e) != LST_OK) return LST_E_STATE;
  const int *c = e->ctr();
  const lst::Ws &w = e->ws();
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
    std::vector<int2> v; std::vector<float2> bb;
    HIP_TRY(d2h(v, w.ls_md, n)); HIP_TRY(d2h(bb, w.ls_beta, n));
    k = 2; mds.resize(2 * (size_t)n);
    for (int i = 0; i < n; ++i) { mds[2 * i] = v[i].x; mds[2 * i + 1] = v[i].y; a[2 * i] = bb[i].x; a[2 * i + 1] = bb[i].y; }
  } else if (stage == 2) {
    std::vector<int4> v; std::vector<float4> bb;
    HIP_TRY(d2h(v, w.t3_md, n)); HIP_TRY(d2h(bb, w.t3_attr, n));
    k = 3; mds.resize(3 * (size_t)n);
    for (int i = 0; i < n; ++i) {
      mds[3 * i] = v[i].x; mds[3 * i + 1] = v[i].y; mds[3 * i + 2] = v[i].z;
      a[4 * i] = bb[i].x; a[4 * i + 1] = bb[i].y; a[4 * i + 2] = bb[i].z; a[4 * i + 3] = bb[i].w;
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
    std::vector<int2> so; std::vector<float4> bb;
    HIP_TRY(d2h(so, five ? (const void *)w.pt5_so : (const void *)w.pt3_so, n));
    HIP_TRY(d2h(bb, five ? (const void *)w.pt5_attr : (const void *)w.pt3_attr, n));
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
      a[3 * i] = bb[i].x; a[3 * i + 1] = bb[i].y; a[3 * i + 2] = bb[i].z;
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

lst_status lst_release_event(lst_event e);

// ------------------------------------------------------------------ plans
struct lst_plan_s {
  lst_geometry geom = nullptr;
  int B = 0, max_hits = 0, max_seeds = 0;
  lst::Caps caps{};
  char *base = nullptr;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  lst_batch_s *pending = nullptr;  // the last run, until all its events are released
};

static size_t plan_bytes(int n_mod, int B, int max_hits, int max_seeds, const lst::Caps &c) {
  return header_bytes(B) +
         (size_t)B * lst::workspace_layout(n_mod, max_hits, max_seeds, c, nullptr, nullptr, nullptr);
}

lst_status lst_plan_workspace_bytes(lst_geometry g, int32_t B, int32_t max_hits, int32_t max_seeds,
                                    const lst_capacity *cap, size_t *bytes) {
  if (!g || !bytes || B < 1 || B > 65535) return fail(LST_E_INVALID, "lst_plan_workspace_bytes: bad argument");
  std::vector<lst::Caps> c;
  lst_status s = resolve_caps(1, &max_hits, &max_seeds, cap, c);
  if (s != LST_OK) return s;
  *bytes = plan_bytes(g->g.n_mod, B, max_hits, max_seeds, c[0]);
  return LST_OK;
}

// Descriptor of slot i of a plan holding event `ev` (NULL = empty slot).
static void plan_slot(const lst_plan_s *p, int i, const lst_event_desc *ev, lst::Ws *w) {
  const size_t slot = lst::workspace_layout(p->geom->g.n_mod, p->max_hits, p->max_seeds, p->caps, nullptr, nullptr,
                                            nullptr);
  int *d_ctr = reinterpret_cast<int *>(p->base + ((sizeof(lst::Ws) * (size_t)p->B + kAlign - 1) / kAlign) * kAlign);
  const int nh = ev ? ev->n_hits : 0, ns = ev ? ev->n_seeds : 0;
  lst::workspace_layout(p->geom->g.n_mod, nh, ns, p->caps, w, p->base + header_bytes(p->B) + slot * i,
                        d_ctr + (size_t)i * lst::C_COUNT, p->max_hits, p->max_seeds);
  if (ev) {
    w->x = ev->x; w->y = ev->y; w->z = ev->z; w->module = ev->module; w->sensor = ev->sensor;
    w->px = ev->px; w->py = ev->py; w->pz = ev->pz; w->q = ev->q; w->hits4 = ev->hits4;
  }
}

lst_status lst_plan_create(lst_geometry g, int32_t B, int32_t max_hits, int32_t max_seeds, const lst_capacity *cap,
                           void *workspace, size_t ws_bytes, void *stream, lst_plan *out) {
  if (!out) return fail(LST_E_INVALID, "lst_plan_create: NULL out");
  *out = nullptr;
  if (!g || !workspace || B < 1 || B > 65535) return fail(LST_E_INVALID, "lst_plan_create: bad argument");
  if (max_hits < 0) return fail(LST_E_INVALID, "lst_plan_create: negative max_hits");
  lst_status bs = check_bucketing(g, max_hits);
  if (bs != LST_OK) return bs;
  std::vector<lst::Caps> c;
  lst_status s = resolve_caps(1, &max_hits, &max_seeds, cap, c);
  if (s != LST_OK) return s;
  const size_t need = plan_bytes(g->g.n_mod, B, max_hits, max_seeds, c[0]);
  if (ws_bytes < need) return fail(LST_E_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return fail(LST_E_INVALID, "workspace not 256-byte aligned");
  auto *p = new (std::nothrow) lst_plan_s();
  if (!p) return fail(LST_E_NOMEM, "host allocation failed");
  p->geom = g; p->B = B; p->max_hits = max_hits; p->max_seeds = max_seeds; p->caps = c[0];
  p->base = reinterpret_cast<char *>(workspace);
  p->stream = reinterpret_cast<hipStream_t>(stream);
  // launch grids of the captured chain follow the slot bounds
  lst::Ws bound{};
  plan_slot(p, 0, nullptr, &bound);
  bound.n_hits = max_hits;
  bound.n_seeds = max_seeds;
  bound.cap_tc = (int)(c[0].pt5 + c[0].pt3 + c[0].t5 + max_seeds);
  const lst::Ws *d_ws = reinterpret_cast<const lst::Ws *>(p->base);
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    lst::enqueue_chain(g->g, d_ws, B, bound, cs, nullptr, g->site_block);
    hipError_t le = hipGetLastError();
    e = hipStreamEndCapture(cs, &p->graph);
    if (e == hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (cs) drop(hipStreamDestroy(cs));
  if (e != hipSuccess) {
    if (p->exec) drop(hipGraphExecDestroy(p->exec));
    if (p->graph) drop(hipGraphDestroy(p->graph));
    delete p;
    return fail(LST_E_DEVICE, std::string("lst_plan_create: graph capture failed: ") + hipGetErrorString(e));
  }
  *out = p;
  return LST_OK;
}

lst_status lst_plan_run(lst_plan p, int32_t n_events, const lst_event_desc *evs, void *stream, lst_event *out) {
  if (!p || !out || n_events < 0 || n_events > p->B || (n_events > 0 && !evs))
    return fail(LST_E_INVALID, "lst_plan_run: bad argument");
  for (int i = 0; i < n_events; ++i) {
    out[i] = nullptr;
    const lst_event_desc &ev = evs[i];
    if (ev.n_hits < 0 || ev.n_seeds < 0 || ev.n_hits > p->max_hits || ev.n_seeds > p->max_seeds)
      return fail(LST_E_INVALID, "event larger than the plan's slots");
    if (ev.n_hits > 0 && (!ev.x || !ev.y || !ev.z || !ev.module || !ev.sensor))
      return fail(LST_E_INVALID, "hit arrays missing");
    if (ev.n_seeds > 0 && (!ev.px || !ev.py || !ev.pz || !ev.q || !ev.hits4))
      return fail(LST_E_INVALID, "seed arrays missing");
  }
  if (p->pending) return fail(LST_E_STATE, "events of the previous run of this plan are still held");
  auto *b = new (std::nothrow) lst_batch_s();
  if (!b) return fail(LST_E_NOMEM, "host allocation failed");
  b->geom = p->geom;
  b->B = p->B;
  b->stream = stream ? reinterpret_cast<hipStream_t>(stream) : p->stream;
  b->refs = 1;  // creation reference, dropped at the end of this call
  if (!batch_host_resources(b, p->B)) {
    release_batch_ref(b);
    return fail(LST_E_DEVICE, "lst_plan_run: pinned buffers or event creation failed");
  }
  for (int i = 0; i < p->B; ++i) plan_slot(p, i, i < n_events ? &evs[i] : nullptr, &b->h_ws[i]);
  int *d_ctr = reinterpret_cast<int *>(p->base + ((sizeof(lst::Ws) * (size_t)p->B + kAlign - 1) / kAlign) * kAlign);
  hipError_t he = hipMemcpyAsync(p->base, b->h_ws, sizeof(lst::Ws) * p->B, hipMemcpyHostToDevice, b->stream);
  if (he == hipSuccess) he = hipGraphLaunch(p->exec, b->stream);
  if (he == hipSuccess)
    he = hipMemcpyAsync(b->h_ctr, d_ctr, sizeof(int) * lst::C_COUNT * p->B, hipMemcpyDeviceToHost, b->stream);
  if (he == hipSuccess) he = hipEventRecord(b->done, b->stream);
  if (he != hipSuccess) b->failed = true;
  for (int i = 0; i < n_events; ++i) {
    auto *e = new (std::nothrow) lst_event_s();
    if (!e) {
      for (int k = 0; k < i; ++k) { lst_release_event(out[k]); out[k] = nullptr; }
      release_batch_ref(b);
      return fail(LST_E_NOMEM, "host allocation failed");
    }
    e->batch = b;
    e->index = i;
    ++b->refs;
    out[i] = e;
  }
  // The events' objects live in the plan's workspace: the next run is refused
  // until every event of this one has been released (which waits for it).
  b->owner = &p->pending;
  p->pending = b;
  release_batch_ref(b);
  if (he != hipSuccess) return fail(LST_E_DEVICE, std::string("lst_plan_run: ") + hipGetErrorString(he));
  return LST_OK;
}

lst_status lst_plan_release(lst_plan p) {
  if (!p) return LST_OK;
  if (p->pending) p->pending->owner = nullptr;
  if (p->exec) drop(hipGraphExecDestroy(p->exec));
  if (p->graph) drop(hipGraphDestroy(p->graph));
  delete p;
  return LST_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ server
namespace {

struct SrvReq {
  int64_t id;
  lst_event_desc ev;
  double arrival;
  size_t region;  // footprint of the event's region in a batch workspace
  lst::Caps caps;  // object capacities of the next attempt
  int attempts;    // runs that overflowed a capacity so far
};
constexpr int kSrvMaxAttempts = 4;  // a request whose capacities grew this often is reported as failed

struct SrvFlight {
  lst_batch_s *batch;
  std::vector<SrvReq> reqs;
  double admit;
  int stream;
};

double secs_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct lst_server_s {
  lst_geometry geom = nullptr;
  lst_server_config cfg{};
  int device = 0;
  char *pool = nullptr;
  size_t pool_bytes = 0;
  std::map<size_t, size_t> free_blocks;  // offset -> size, coalesced
  std::map<size_t, size_t> used_blocks;  // offset -> size
  std::vector<hipStream_t> streams;
  std::mutex mu;  // guards pending, results, the allocator, live, counters
  std::deque<SrvReq> pending;
  std::vector<lst_server_result> results;
  std::map<lst_batch_s *, int> live;  // batches whose events are out with the client
  std::vector<SrvFlight> flights;     // scheduler thread only
  std::thread th;
  std::condition_variable cv;  // wakes the idle scheduler: a submission, a released batch, stop
  std::atomic<bool> stop{false};
  std::chrono::steady_clock::time_point t0;
  int64_t n_batches = 0;
  int64_t n_reruns = 0;  // requests run again after a capacity overflow
};

// caller holds s->mu
static void server_free_block_locked(lst_server_s *s, size_t off) {
  auto it = s->used_blocks.find(off);
  if (it == s->used_blocks.end()) return;
  size_t size = it->second;
  s->used_blocks.erase(it);
  auto nx = s->free_blocks.lower_bound(off);
  if (nx != s->free_blocks.end() && off + size == nx->first) {
    size += nx->second;
    nx = s->free_blocks.erase(nx);
  }
  if (nx != s->free_blocks.begin()) {
    auto pv = std::prev(nx);
    if (pv->first + pv->second == off) {
      pv->second += size;
      return;
    }
  }
  s->free_blocks.emplace(off, size);
}

static void server_free_block(lst_server_s *s, size_t off) {
  std::lock_guard<std::mutex> lk(s->mu);
  server_free_block_locked(s, off);
}

// a server batch's last event was released: its workspace block returns to the pool
static void server_release_batch(lst_server_s *s, lst_batch_s *b) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->live.erase(b);
    server_free_block_locked(s, b->block_off);
  }
  s->cv.notify_one();  // pending requests may fit now
}

// Capacities of a rerun after an overflow: every stage at least 1.5 x its
// required count (required counts are exact up to the stage that overflowed
// and lower bounds after it), clamped to the device scans' limit.
static lst::Caps grown_caps(const lst::Caps &c, const int *ctr) {
  auto grow = [](int64_t cur, int req) {
    const int64_t want = std::max<int64_t>(cur, (int64_t)req + req / 2 + 1024);
    return std::min<int64_t>(want, kMaxCap);
  };
  lst::Caps g = c;
  g.md = grow(c.md, ctr[lst::C_RMD]);
  g.ls = grow(c.ls, ctr[lst::C_RLS]);
  g.t3 = grow(c.t3, ctr[lst::C_RT3]);
  g.t5 = grow(c.t5, ctr[lst::C_RT5]);
  g.pt3 = grow(c.pt3, ctr[lst::C_RPT3]);
  g.pt5 = grow(c.pt5, ctr[lst::C_RPT5]);
  return g;
}

// first fit; caller holds s->mu; returns SIZE_MAX when nothing fits
static size_t server_alloc(lst_server_s *s, size_t size) {
  size = (size + kAlign - 1) / kAlign * kAlign;
  for (auto it = s->free_blocks.begin(); it != s->free_blocks.end(); ++it) {
    if (it->second < size) continue;
    const size_t off = it->first, rest = it->second - size;
    s->free_blocks.erase(it);
    if (rest) s->free_blocks.emplace(off + size, rest);
    s->used_blocks.emplace(off, size);
    return off;
  }
  return SIZE_MAX;
}

static void server_loop(lst_server_s *s) {
  (void)hipSetDevice(s->device);
  std::vector<int> busy(s->streams.size(), 0);
  while (!s->stop.load() || !s->flights.empty()) {
    bool worked = false;
    // completions
    for (size_t f = 0; f < s->flights.size();) {
      SrvFlight &fl = s->flights[f];
      const hipError_t q = fl.batch->failed ? hipErrorUnknown : hipEventQuery(fl.batch->done);
      if (q == hipErrorNotReady) { ++f; continue; }
      const double t = secs_since(s->t0);
      fl.batch->synced = true;
      std::vector<lst_event> evs(fl.reqs.size(), nullptr);
      make_events(fl.batch, (int)fl.reqs.size(), evs.data());
      std::vector<lst_event> rerun_evs;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        s->live[fl.batch] = 1;
        std::vector<SrvReq> rerun;
        for (size_t i = 0; i < fl.reqs.size(); ++i) {
          lst_server_result r{};
          r.id = fl.reqs[i].id;
          r.event = evs[i];
          r.arrival_s = fl.reqs[i].arrival;
          r.admit_s = fl.admit;
          r.done_s = t;
          const int *ctr = fl.batch->h_ctr + i * lst::C_COUNT;
          const int st = ctr[lst::C_STATUS];
          r.status = fl.batch->failed ? LST_E_DEVICE
                     : (st & (lst::ST_BAD_HIT | lst::ST_BAD_SEED)) ? LST_E_INVALID
                     : (st & lst::ST_CAPACITY) ? LST_E_CAPACITY : LST_OK;
          if (r.status == LST_E_CAPACITY && fl.reqs[i].attempts + 1 < kSrvMaxAttempts) {
            // grow the capacities from the required counts and run the request again, ahead of
            // the queue (its arrival time, hence its latency, is kept)
            SrvReq q = fl.reqs[i];
            q.caps = grown_caps(q.caps, ctr);
            q.attempts += 1;
            q.region = lst::workspace_layout(s->geom->g.n_mod, q.ev.n_hits, q.ev.n_seeds, q.caps, nullptr, nullptr,
                                             nullptr);
            const bool scan_ok = q.caps.pt5 + q.caps.pt3 + q.caps.t5 + q.ev.n_seeds <= kMaxTc;
            if (!scan_ok) {
              s->results.push_back(r);  // the grown capacities would exceed the candidates' scan
              continue;
            }
            if (q.region + header_bytes(1) <= s->pool_bytes) {
              rerun.push_back(q);
              rerun_evs.push_back(evs[i]);
              ++s->n_reruns;
              continue;
            }
            r.status = LST_E_NOMEM;  // the grown event no longer fits the pool
          }
          s->results.push_back(r);
        }
        for (auto it = rerun.rbegin(); it != rerun.rend(); ++it) s->pending.push_front(*it);
      }
      for (lst_event e : rerun_evs) lst_release_event(e);  // may free the batch's block (takes s->mu)
      busy[fl.stream] = 0;
      s->flights.erase(s->flights.begin() + (long)f);
      worked = true;
    }
    // admission: arrived requests, FIFO, batched, as streams and pool memory allow
    for (size_t si = 0; si < s->streams.size() && !s->stop.load(); ++si) {
      if (busy[si]) continue;
      const double now = secs_since(s->t0);
      std::vector<SrvReq> take;
      size_t off = SIZE_MAX;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        size_t k = 0;
        while (k < s->pending.size() && (int)k < s->cfg.max_batch && s->pending[k].arrival <= now) ++k;
        while (k > 0) {
          size_t need = header_bytes((int)k);
          for (size_t i = 0; i < k; ++i) need += s->pending[i].region;
          off = server_alloc(s, need);
          if (off != SIZE_MAX) break;
          --k;
        }
        for (size_t i = 0; i < k; ++i) {
          take.push_back(s->pending.front());
          s->pending.pop_front();
        }
      }
      if (take.empty()) break;
      std::vector<lst_event_desc> evs(take.size());
      std::vector<int32_t> nh(take.size()), ns(take.size());
      for (size_t i = 0; i < take.size(); ++i) {
        evs[i] = take[i].ev;
        nh[i] = evs[i].n_hits;
        ns[i] = evs[i].n_seeds;
      }
      std::vector<lst::Caps> caps(take.size());
      for (size_t i = 0; i < take.size(); ++i) caps[i] = take[i].caps;
      lst_batch_s *b = nullptr;
      enqueue_batch_at(s->geom, (int)take.size(), evs.data(), caps, s->pool + off, s->streams[si], &b);
      if (!b) {  // host allocation failure: report the requests as failed
        server_free_block(s, off);
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto &r : take) {
          lst_server_result res{};
          res.id = r.id; res.arrival_s = r.arrival; res.admit_s = now; res.done_s = now; res.status = LST_E_NOMEM;
          s->results.push_back(res);
        }
        continue;
      }
      b->server = s;
      b->block_off = off;
      s->flights.push_back(SrvFlight{b, std::move(take), now, (int)si});
      busy[si] = 1;
      ++s->n_batches;
      worked = true;
    }
    if (!worked) {
      if (!s->flights.empty()) {
        std::this_thread::yield();  // batches in flight: poll their completion events
        continue;
      }
      // idle: sleep until a submission, a released batch, stop, or the next arrival
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop.load()) continue;
      double next = -1.0;
      for (const auto &q : s->pending) next = next < 0 ? q.arrival : std::min(next, q.arrival);
      const double now = secs_since(s->t0);
      if (next < 0) {
        s->cv.wait_for(lk, std::chrono::milliseconds(50));
      } else if (next > now) {
        s->cv.wait_for(lk, std::chrono::duration<double>(std::min(next - now, 0.05)));
      } else if (!s->live.empty()) {
        // arrived requests waiting for pool memory held by results the client still has
        s->cv.wait_for(lk, std::chrono::milliseconds(1));
      }
    }
  }
}

extern "C" {

lst_status lst_server_create(lst_geometry g, const lst_server_config *cfg, void *pool, size_t pool_bytes,
                             lst_server *out) {
  if (!out) return fail(LST_E_INVALID, "lst_server_create: NULL out");
  *out = nullptr;
  if (!g || !cfg || !pool || cfg->n_streams < 1 || cfg->n_streams > 64 || cfg->max_batch < 1 ||
      cfg->max_batch > 1024)
    return fail(LST_E_INVALID, "lst_server_create: bad argument");
  if (reinterpret_cast<uintptr_t>(pool) % kAlign != 0) return fail(LST_E_INVALID, "pool not 256-byte aligned");
  auto *s = new (std::nothrow) lst_server_s();
  if (!s) return fail(LST_E_NOMEM, "host allocation failed");
  s->geom = g;
  s->cfg = *cfg;
  s->pool = reinterpret_cast<char *>(pool);
  s->pool_bytes = pool_bytes / kAlign * kAlign;
  s->free_blocks.emplace(0, s->pool_bytes);
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return fail(LST_E_DEVICE, "hipGetDevice failed");
  }
  for (int i = 0; i < cfg->n_streams; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) drop(hipStreamDestroy(x));
      delete s;
      return fail(LST_E_DEVICE, "stream creation failed");
    }
    s->streams.push_back(st);
  }
  s->t0 = std::chrono::steady_clock::now();
  s->th = std::thread(server_loop, s);
  *out = s;
  return LST_OK;
}

lst_status lst_server_now(lst_server s, double *t) {
  if (!s || !t) return fail(LST_E_INVALID, "lst_server_now: NULL argument");
  *t = secs_since(s->t0);
  return LST_OK;
}

lst_status lst_server_submit_with_capacity(lst_server s, const lst_event_desc *ev, const lst_capacity *cap,
                                           int64_t id, double arrival_s) {
  if (!s || !ev) return fail(LST_E_INVALID, "lst_server_submit: NULL argument");
  lst_status st = check_event_desc(*ev);
  if (st == LST_OK) st = check_bucketing(s->geom, ev->n_hits);
  if (st != LST_OK) return st;
  std::vector<lst::Caps> caps;
  st = resolve_caps(1, &ev->n_hits, &ev->n_seeds, cap, caps);
  if (st != LST_OK) return st;
  const size_t region = lst::workspace_layout(s->geom->g.n_mod, ev->n_hits, ev->n_seeds, caps[0], nullptr, nullptr,
                                              nullptr);
  if (region + header_bytes(1) > s->pool_bytes) return fail(LST_E_NOMEM, "event larger than the server's pool");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->pending.push_back(SrvReq{id, *ev, arrival_s, region, caps[0], 0});
  }
  s->cv.notify_one();
  return LST_OK;
}

lst_status lst_server_submit(lst_server s, const lst_event_desc *ev, int64_t id, double arrival_s) {
  return lst_server_submit_with_capacity(s, ev, nullptr, id, arrival_s);
}

lst_status lst_server_reruns(lst_server s, int64_t *n) {
  if (!s || !n) return fail(LST_E_INVALID, "lst_server_reruns: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *n = s->n_reruns;
  return LST_OK;
}

lst_status lst_server_poll(lst_server s, lst_server_result *out, int32_t max, int32_t *n) {
  if (!s || !n || (max > 0 && !out)) return fail(LST_E_INVALID, "lst_server_poll: bad argument");
  std::lock_guard<std::mutex> lk(s->mu);
  const int k = std::min<int>(max, (int)s->results.size());
  for (int i = 0; i < k; ++i) out[i] = s->results[i];
  s->results.erase(s->results.begin(), s->results.begin() + k);
  *n = k;
  return LST_OK;
}

lst_status lst_server_pending(lst_server s, int32_t *queued, int32_t *ready) {
  if (!s || !queued || !ready) return fail(LST_E_INVALID, "lst_server_pending: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *queued = (int32_t)s->pending.size();
  *ready = (int32_t)s->results.size();
  return LST_OK;
}

lst_status lst_server_destroy(lst_server s) {
  if (!s) return LST_OK;
  s->stop.store(true);
  s->cv.notify_all();
  if (s->th.joinable()) s->th.join();  // returns once in-flight batches completed
  std::vector<lst_server_result> left;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    left.swap(s->results);
  }
  for (auto &r : left)
    if (r.event) lst_release_event(r.event);
  {
    // batches whose events the client still holds no longer return memory here
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &kv : s->live) kv.first->server = nullptr;
  }
  for (auto st : s->streams) drop(hipStreamDestroy(st));
  delete s;
  return LST_OK;
}

// ---------------------------------------------------------------- launch shapes
lst_status lst_get_launch_config(lst_geometry g, int32_t n, int32_t *site_block) {
  if (!g || !site_block || n < lst::kNumSites) return fail(LST_E_INVALID, "lst_get_launch_config: bad argument");
  for (int s = 0; s < lst::kNumSites; ++s)
    site_block[s] = lst::site_tunable(s) ? (g->site_block[s] > 0 ? g->site_block[s] : 256) : 0;
  return LST_OK;
}

static bool valid_block(int s, int b) {
  return lst::site_tunable(s) ? (b == 0 || b == 64 || b == 128 || b == 256) : b == 0;
}

lst_status lst_set_launch_config(lst_geometry g, int32_t n, const int32_t *site_block) {
  if (!g || !site_block || n != lst::kNumSites) return fail(LST_E_INVALID, "lst_set_launch_config: bad argument");
  for (int s = 0; s < n; ++s)
    if (!valid_block(s, site_block[s]))
      return fail(LST_E_INVALID, std::string("lst_set_launch_config: site ") + lst::kSiteNames[s] +
                                     " takes 0 (default)" + (lst::site_tunable(s) ? ", 64, 128 or 256" : " only"));
  for (int s = 0; s < n; ++s) g->site_block[s] = site_block[s];
  return LST_OK;
}

lst_status lst_autotune(lst_geometry g, int32_t B, const lst_event_desc *evs, const lst_capacity *cap, void *workspace,
                        size_t ws_bytes, void *stream, int32_t reps, float *site_ms) {
  if (!g || !evs || !workspace || B < 1 || B > 65535 || reps < 1 || reps > 100)
    return fail(LST_E_INVALID, "lst_autotune: bad argument");
  std::vector<int32_t> nh(B), ns(B);
  for (int i = 0; i < B; ++i) {
    lst_status s = check_event_desc(evs[i]);
    if (s == LST_OK) s = check_bucketing(g, evs[i].n_hits);
    if (s != LST_OK) return s;
    nh[i] = evs[i].n_hits;
    ns[i] = evs[i].n_seeds;
  }
  std::vector<lst::Caps> caps;
  lst_status s = resolve_caps(B, nh.data(), ns.data(), cap, caps);
  if (s != LST_OK) return s;
  if (ws_bytes < batch_bytes(g->g.n_mod, B, nh.data(), ns.data(), caps))
    return fail(LST_E_NOMEM, "lst_autotune: workspace too small (see lst_batch_workspace_bytes)");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return fail(LST_E_INVALID, "workspace not 256-byte aligned");
  if (site_ms)
    for (int k = 0; k < lst::kNumSites; ++k) site_ms[k] = -1.0f;
  int saved[lst::kMaxSites];
  std::copy(g->site_block, g->site_block + lst::kMaxSites, saved);
  auto restore = [&](lst_status st) {
    std::copy(saved, saved + lst::kMaxSites, g->site_block);
    return st;
  };
  // one timed batch with the current launch shapes: the site's launch time, or an error
  auto time_site = [&](int site, float *ms) -> lst_status {
    lst_batch_s *b = nullptr;
    lst_status es = enqueue_batch_at(g, B, evs, caps, reinterpret_cast<char *>(workspace),
                                     reinterpret_cast<hipStream_t>(stream), &b, site);
    if (!b) return es;
    lst_status rs = es;
    if (rs == LST_OK) {
      hipError_t e = hipEventSynchronize(b->done);
      if (e == hipSuccess) {
        b->synced = true;
        e = hipEventElapsedTime(ms, b->tbeg, b->tend);
      }
      if (e != hipSuccess) rs = fail(LST_E_DEVICE, std::string("lst_autotune: ") + hipGetErrorString(e));
      for (int i = 0; i < B && rs == LST_OK; ++i) rs = map_status(b->h_ctr[(size_t)i * lst::C_COUNT + lst::C_STATUS]);
    }
    for (int i = 0; i < B; ++i) release_batch_ref(b);
    return rs;
  };
  const int choices[3] = {64, 128, 256};
  for (int site = 0; site < lst::kNumSites; ++site) {
    if (!lst::site_tunable(site)) continue;
    float best = 3.0e38f;
    int best_b = g->site_block[site];
    for (int c : choices) {
      g->site_block[site] = c;
      float tmin = 3.0e38f;
      for (int r = 0; r < reps; ++r) {
        float ms = 0.0f;
        lst_status ts = time_site(site, &ms);
        if (ts != LST_OK) return restore(ts);
        tmin = std::min(tmin, ms);
      }
      if (tmin < best) {
        best = tmin;
        best_b = c;
      }
    }
    g->site_block[site] = best_b;
    if (site_ms) site_ms[site] = best;
  }
  return LST_OK;
}

// ------------------------------------------------------------------ tiles
namespace {
struct TileSpec {
  const char *name;
  int lo, hi;
  int choices[4];  // autotuner candidates, 0-terminated (0 may also be a choice: listed first)
  int n_choices;
};
const TileSpec kTileSpecs[] = {
    {"md_cache", 0, lst::kMdCache, {0, 16, lst::kMdCache}, 3},
    {"ls_cache", 0, lst::kLsCache, {8, 16, lst::kLsCache}, 3},
    {"t3_cache", 0, lst::kT3Cache, {0, 1, 2}, 3},
    {"t5_cache", 0, lst::kT5Cache, {0, 1, 2}, 3},
    {"pt3_cache", 0, lst::kPt3Cache, {64, 128, lst::kPt3Cache}, 3},
    {"pt5_cache", 0, lst::kPt5Cache, {4, 8, lst::kPt5Cache}, 3},
    {"pass_list", 1, lst::kPassList, {256, lst::kPassList}, 2},
    {"max_slices", 1, lst::kMaxSlices, {128, lst::kMaxSlices}, 2},
    {"ext_per_wave", 4, 16, {4, 8, 16}, 3},
    {"ls_group", 0, lst::kLsGroup, {0, 1, lst::kLsGroup}, 3},
};
constexpr int kNumTiles = (int)(sizeof(kTileSpecs) / sizeof(kTileSpecs[0]));
int *tile_field(lst::Tiles &t, int i) {
  int *f[kNumTiles] = {&t.md_cache, &t.ls_cache, &t.t3_cache, &t.t5_cache, &t.pt3_cache,
                       &t.pt5_cache, &t.pass_list, &t.max_slices, &t.ext_per_wave, &t.ls_group};
  return f[i];
}
bool tile_ok(int i, int v) {
  if (v < kTileSpecs[i].lo || v > kTileSpecs[i].hi) return false;
  return i != 8 || v == 4 || v == 8 || v == 16;  // the extension search is built for these
}
}  // namespace

int32_t lst_tile_count(void) { return kNumTiles; }

const char *lst_tile_name(int32_t i) { return (i >= 0 && i < kNumTiles) ? kTileSpecs[i].name : nullptr; }

lst_status lst_tile_range(int32_t i, int32_t *lo, int32_t *hi) {
  if (i < 0 || i >= kNumTiles || !lo || !hi) return fail(LST_E_INVALID, "lst_tile_range: bad argument");
  *lo = kTileSpecs[i].lo;
  *hi = kTileSpecs[i].hi;
  return LST_OK;
}

lst_status lst_get_tile_config(lst_geometry g, int32_t n, int32_t *tiles) {
  if (!g || !tiles || n != kNumTiles) return fail(LST_E_INVALID, "lst_get_tile_config: bad argument");
  for (int i = 0; i < kNumTiles; ++i) tiles[i] = *tile_field(g->g.tiles, i);
  return LST_OK;
}

lst_status lst_set_tile_config(lst_geometry g, int32_t n, const int32_t *tiles) {
  if (!g || !tiles || n != kNumTiles) return fail(LST_E_INVALID, "lst_set_tile_config: bad argument");
  for (int i = 0; i < kNumTiles; ++i)
    if (!tile_ok(i, tiles[i])) {
      char msg[160];
      snprintf(msg, sizeof(msg), "lst_set_tile_config: %s = %d outside [%d, %d]%s", kTileSpecs[i].name, tiles[i],
               kTileSpecs[i].lo, kTileSpecs[i].hi, i == 8 ? " or not 4, 8, 16" : "");
      return fail(LST_E_INVALID, msg);
    }
  for (int i = 0; i < kNumTiles; ++i) *tile_field(g->g.tiles, i) = tiles[i];
  return LST_OK;
}

lst_status lst_autotune_tiles(lst_geometry g, int32_t B, const lst_event_desc *evs, const lst_capacity *cap,
                              void *workspace, size_t ws_bytes, void *stream, int32_t reps, float *tile_ms) {
  if (!g || !evs || !workspace || B < 1 || B > 65535 || reps < 1 || reps > 100)
    return fail(LST_E_INVALID, "lst_autotune_tiles: bad argument");
  std::vector<int32_t> nh(B), ns(B);
  for (int i = 0; i < B; ++i) {
    lst_status s = check_event_desc(evs[i]);
    if (s == LST_OK) s = check_bucketing(g, evs[i].n_hits);
    if (s != LST_OK) return s;
    nh[i] = evs[i].n_hits;
    ns[i] = evs[i].n_seeds;
  }
  std::vector<lst::Caps> caps;
  lst_status s = resolve_caps(B, nh.data(), ns.data(), cap, caps);
  if (s != LST_OK) return s;
  if (ws_bytes < batch_bytes(g->g.n_mod, B, nh.data(), ns.data(), caps))
    return fail(LST_E_NOMEM, "lst_autotune_tiles: workspace too small (see lst_batch_workspace_bytes)");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return fail(LST_E_INVALID, "workspace not 256-byte aligned");
  const lst::Tiles saved = g->g.tiles;
  // one timed batch with the current tiles: the whole chain's time, or an error
  auto time_chain = [&](float *ms) -> lst_status {
    lst_batch_s *b = nullptr;
    lst_status es = enqueue_batch_at(g, B, evs, caps, reinterpret_cast<char *>(workspace),
                                     reinterpret_cast<hipStream_t>(stream), &b, lst::kChainSite);
    if (!b) return es;
    lst_status rs = es;
    if (rs == LST_OK) {
      hipError_t e = hipEventSynchronize(b->done);
      if (e == hipSuccess) {
        b->synced = true;
        e = (b->tbeg && b->tend) ? hipEventElapsedTime(ms, b->tbeg, b->tend) : hipErrorInvalidValue;
      }
      if (e != hipSuccess) rs = fail(LST_E_DEVICE, std::string("lst_autotune_tiles: ") + hipGetErrorString(e));
      for (int i = 0; i < B && rs == LST_OK; ++i) rs = map_status(b->h_ctr[(size_t)i * lst::C_COUNT + lst::C_STATUS]);
    }
    for (int i = 0; i < B; ++i) release_batch_ref(b);
    return rs;
  };
  for (int t = 0; t < kNumTiles; ++t) {
    if (tile_ms) tile_ms[t] = -1.0f;
    if (t == 8 && !g->g.ext) continue;  // the extension search runs only with extensions on
    float best = 3.0e38f;
    int best_v = *tile_field(g->g.tiles, t);
    for (int c = 0; c < kTileSpecs[t].n_choices; ++c) {
      *tile_field(g->g.tiles, t) = kTileSpecs[t].choices[c];
      float tmin = 3.0e38f;
      for (int r = 0; r < reps; ++r) {
        float ms = 0.0f;
        lst_status ts = time_chain(&ms);
        if (ts != LST_OK) {
          g->g.tiles = saved;
          return ts;
        }
        tmin = std::min(tmin, ms);
      }
      if (tmin < best) {
        best = tmin;
        best_v = kTileSpecs[t].choices[c];
      }
    }
    *tile_field(g->g.tiles, t) = best_v;
    if (tile_ms) tile_ms[t] = best;
  }
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
  if (event_ok(e) != LST_OK) return LST_E_STATE;
  if (e->batch->timed_site < 0) return fail(LST_E_STATE, "no launch site was timed for this event");
  HIP_TRY(hipEventElapsedTime(ms, e->batch->tbeg, e->batch->tend));
  return LST_OK;
}

lst_status lst_release_event(lst_event e) {
  if (!e) return LST_OK;
  release_batch_ref(e->batch);
  delete e;
  return LST_OK;
}

}  // extern "C"
