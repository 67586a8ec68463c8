// gfx950 kernels of the Line Segment Tracking chain (arXiv:2207.08207).
//
// Every stage follows one pattern: count objects per parent (module, MD, LS,
// T3, seed), exclusive-scan the counts on the device, then fill each parent's
// objects at its scanned offset in a fixed order.  No global atomics decide
// an output position, so the object arrays are identical run to run; the
// only atomics are histogram counts and the scatter into per-MD / per-hit
// incidence lists, whose consumers are order-independent.  Object counts
// stay on the device: later kernels read them and stride over them, so the
// whole chain is enqueued without a host round trip.
#include <hip/hip_fp16.h>

#include <cstring>
#include <type_traits>

#include "lst_select.hpp"
#include "lst_ws.hpp"

namespace lst {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kScanItems = 8;                       // per thread
constexpr int kScanTile = kBlock * kScanItems;      // per block
constexpr int kMaxScanBlocks = 4096;                // tile sums a scan keeps (scan_tmp): n < 8M
static_assert((long)kMaxScanBlocks * kScanTile > 8000000L, "scan of the largest count of an event");

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
// Set bits of a ballot below this lane (its rank among the set lanes).
__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Wave-uniform values in scalar registers: the compiler cannot prove a value
// derived from threadIdx.x, or loaded through a generic pointer, uniform, and
// would otherwise keep it (and every address computed from it) in vector
// registers.  uload is for loads whose address is the same on every lane.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }
__device__ __forceinline__ int uload(const int *p) { return __builtin_amdgcn_readfirstlane(*p); }
// The same pointer in the global address space: the workspace and geometry
// pointers are read from memory, so the compiler cannot infer their address
// space and would issue flat loads, which also count against the LDS wait
// counter (every LDS wait then waits for the gathers in flight too) and take a
// 64-bit address per lane.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T *gp(const T *p) {
  return (const __attribute__((address_space(1))) T *)p;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gp(T *p) {
  return (__attribute__((address_space(1))) T *)p;
}
// Loads and stores of vector types through the global address space (their
// member operators take a generic `this`): by their bits, as native vectors.
template <int N> struct NativeOf;
template <> struct NativeOf<4> { typedef int type; };
template <> struct NativeOf<8> { typedef int type __attribute__((ext_vector_type(2))); };
template <> struct NativeOf<16> { typedef int type __attribute__((ext_vector_type(4))); };
template <class T>
__device__ __forceinline__ T gload(const T *p, long i) {
  typedef typename NativeOf<sizeof(T)>::type N;
  const N n = ((const __attribute__((address_space(1))) N *)p)[i];
  T v;
  __builtin_memcpy(&v, &n, sizeof(T));
  return v;
}
template <class T>
__device__ __forceinline__ void gstore(T *p, long i, const T &v) {
  typedef typename NativeOf<sizeof(T)>::type N;
  N n;
  __builtin_memcpy(&n, &v, sizeof(T));
  ((__attribute__((address_space(1))) N *)p)[i] = n;
}

__device__ __forceinline__ int block_sum(int v, int *s_red) {
  // wave reduction by shuffles, then across waves in LDS
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane_id() == 0) s_red[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) t += s_red[w];
  __syncthreads();
  return t;
}

__device__ __forceinline__ int dev_count(const int *p, int fallback) { return p ? *p : fallback; }

// ------------------------------------------------------------------ fill
// Clears the arrays of fill jobs [j0, j1) of every event of the batch.
__global__ void k_clear(const Ws *__restrict__ wb, int j0, int j1) {
  const Ws &w = wb[blockIdx.y];
  for (int j = j0; j < j1; ++j) {
    int *p = w.fills[j].p;
    long n = w.fills[j].n;
    if (w.fills[j].n_dev) n = min(n, (long)w.fills[j].mul * ((long)uload(w.fills[j].n_dev) + 1));
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0;
  }
}

// ------------------------------------------------------------------ scan
// Exclusive scan of in[0..n) into out[0..n], out[n] = total; n = *n_dev (or
// n_fix).  Two passes: tile sums, then each tile's scan offset by the sum of
// the tiles before it.
__global__ void k_scan_reduce(const Ws *__restrict__ wb, int job) {
  __shared__ int s_red[kWaves];
  const Ws &w = wb[blockIdx.y];
  const ScanJob &J = w.scans[job];
  const int n = dev_count(J.n_dev, J.n_fix);
  // tiles 0 .. n / kScanTile (the last one may be empty), strided over the grid
  for (long t = blockIdx.x; t * kScanTile <= n; t += gridDim.x) {
    const long base = t * kScanTile;
    int v = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const long i = base + (long)k * kBlock + threadIdx.x;
      if (i < n) v += J.in[i];
    }
    v = block_sum(v, s_red);
    if (threadIdx.x == 0) w.scan_tmp[t] = v;
  }
}

// Each tile adds the tile sums before it (at most a few hundred for the
// chain's counts) to its own exclusive scan; the tile holding index n writes
// out[n] and the totals.  (Two launches per scan instead of a third,
// single-block pass over the tile sums.)  Both passes stride over the tiles,
// so the grid need not cover the capacity.
__global__ void k_scan_apply(const Ws *__restrict__ wb, int job) {
  __shared__ int s_wave[kWaves], s_red[kWaves];
  const Ws &w = wb[blockIdx.y];
  const ScanJob &J = w.scans[job];
  const int n = dev_count(J.n_dev, J.n_fix);
  for (long t = blockIdx.x; t * kScanTile <= n; t += gridDim.x) {
    const long base = t * kScanTile;
    int pre = 0;
    for (int j = threadIdx.x; j < (int)t; j += blockDim.x) pre += w.scan_tmp[j];
    int run = block_sum(pre, s_red);
    // the tile in kScanItems rounds of kBlock consecutive items
    for (int k = 0; k < kScanItems; ++k) {
      const long i = base + (long)k * kBlock + threadIdx.x;
      const int v = (i < n) ? J.in[i] : 0;
      // inclusive scan within the wave
      int x = v;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane_id() >= o) x += y;
      }
      if (lane_id() == 63) s_wave[threadIdx.x >> 6] = x;
      __syncthreads();
      int wbs = 0, tot = 0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) {
        const int c = s_wave[q];
        wbs += (q < (int)(threadIdx.x >> 6)) ? c : 0;
        tot += c;
      }
      if (i <= n) J.out[i] = run + wbs + x - v;  // out[n] = total
      __syncthreads();
      run += tot;
    }
    if (base + kScanTile > n && threadIdx.x == 0) {
      const int tot = run;  // every item of the later tiles is past n
      if (J.tot_req) *J.tot_req = tot;
      if (J.tot_clamped) {
        *J.tot_clamped = tot < J.cap ? tot : J.cap;
        if (tot > J.cap) atomicOr(w.ctr + C_STATUS, (int)ST_CAPACITY);
      }
    }
  }
}

// blocks for one wave per item (capped; kernels stride)
// Blocks for n items, one wave per item (grid_waves) or one thread per item
// (grid_for), at `block` threads per block; kernels stride over the rest.
static inline int grid_waves(long n, int block = kBlock) {
  const int wpb = block / 64;
  long g = (n + wpb - 1) / wpb;
  if (g < 1) g = 1;
  if (g > 16384) g = 16384;
  return (int)g;
}

// Waves per launch that grid-stride kernels share among the launch's events: eight
// per wave slot of the chip (256 CUs x 32); the searches whose work is a large
// fraction of their capacity (segments, triplets, quintuplets and their
// duplicate removal, MDs) take four times that, since waves with more work
// left than the others hide each other's latency (measured: two per slot made
// the segment count 1.24x slower than eight).
constexpr long kLaunchWaves = 8L * 256 * 32;

static inline int grid_for(long n, int block = kBlock) {
  long g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}

// Scan job `job` of every event of the batch; n_cap bounds the item count.
static void scan(const Ws *wb, int B, int job, long n_cap, hipStream_t st) {
  // tiles covering n_cap + 1 outputs (capacities are checked on the host so that every scan's
  // count stays below kMaxScanBlocks tiles), at most an equal share of kLaunchWaves per event
  const long share = std::max(64L, kLaunchWaves / B / kWaves);
  const int nb = (int)std::min<long>(std::min<long>((n_cap + kScanTile) / kScanTile, kMaxScanBlocks), share);
  k_scan_reduce<<<dim3(nb, B), kBlock, 0, st>>>(wb, job);
  k_scan_apply<<<dim3(nb, B), kBlock, 0, st>>>(wb, job);
}

// ------------------------------------------------------------- windows
__global__ void k_module_windows(const int *info, const float *pos_lo, const float *pos_up, const float *lmin,
                                 const float *lmax, int n_mod, double d0, float4 *win) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n_mod) return;
  double w[4];
  module_windows((info[m] >> 1) & 1, info[m] & 1, (double)pos_lo[m], (double)pos_up[m], (double)lmin[m],
                 (double)lmax[m], d0, w);
  win[m] = make_float4((float)w[0], (float)w[1], (float)w[2], (float)w[3]);
}

void launch_module_windows(const int *info, const float *pos_lo, const float *pos_up, const float *lmin,
                           const float *lmax, int n_mod, double d0, float4 *win, hipStream_t st) {
  k_module_windows<<<(n_mod + 127) / 128, 128, 0, st>>>(info, pos_lo, pos_up, lmin, lmax, n_mod, d0, win);
}

// ------------------------------------------------- allocation-free forms
// One event descriptor written into device memory by a kernel (its argument
// block carries it), for callers that have no host staging buffer.
__global__ void k_put_desc(Ws w, Ws *dst) { *dst = w; }

void launch_put_desc(const Ws &w, Ws *dst, hipStream_t st) { k_put_desc<<<1, 1, 0, st>>>(w, dst); }

// Copies an event's track candidates to caller device buffers: counts[0] =
// candidates, counts[1] = their hits, counts[2] = the chain's status flags;
// the arrays are written only when the chain succeeded and both fit.
__global__ void k_tc_export(const Ws *__restrict__ wb, int max_tc, int max_hits, int *type, int *off, int *hits,
                            int *counts) {
  const Ws &w = wb[0];
  const int st = w.ctr[C_STATUS], n = uload(w.ctr + C_NTC), nh = uload(w.ctr + C_NTCHITS);
  const int tid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
  if (tid == 0) {
    counts[0] = n;
    counts[1] = nh;
    counts[2] = st;
  }
  if (st != 0 || n > max_tc || nh > max_hits) return;
  for (int i = tid; i <= n; i += stride) {
    if (i < n) type[i] = w.tc_type[i];
    off[i] = w.tc_off[i];
  }
  for (int i = tid; i < nh; i += stride) hits[i] = w.tc_hits[i];
}

void launch_tc_export(const Ws *d_ws, int max_tc, int max_hits, int *type, int *off, int *hits, int *counts,
                      hipStream_t st) {
  k_tc_export<<<256, 256, 0, st>>>(d_ws, max_tc, max_hits, type, off, hits, counts);
}

// ------------------------------------------------------------- a0: hits
// Hits are bucketed by key = 2 module + sensor, stably (input order within a
// key), with no global atomic: an LSD-free two-level counting sort.
//  1. k_hits_count: each block counts the hits of its tile of kHitTile input
//     hits per coarse bucket (key >> kFineBits) in LDS and writes the counts,
//     coarse-bucket major (and validates hits and seeds);
//  2. an exclusive scan of those counts gives every (coarse bucket, tile) its
//     first position;
//  3. k_hits_scatter: each wave walks its quarter of the tile again in input
//     order, 64 hits at a time, after the waves before it; hits of one coarse
//     bucket in a round find each other with ballots and take consecutive
//     positions after the bucket's running position (stable), writing one
//     16-byte record (x, y, z, input index and key within the bucket);
//  4. k_bucket_sort: one block per coarse bucket counts its keys, writes their
//     offsets and moves every hit (input index; x, y, z, r) to its key's
//     running position, again 64 hits at a time in order.

// The bucket key of hit i, or -1 for a pixel hit or invalid data (*bad).
__device__ __forceinline__ int hit_key(const Ws &w, int i, int n_mod, bool *bad) {
  const int m = gp(w.module)[i];
  const float x = gp(w.x)[i], y = gp(w.y)[i], z = gp(w.z)[i];
  bool b = !(isfinite(x) && isfinite(y) && isfinite(z)) || m < -1 || m >= n_mod;
  int key = -1;
  if (m >= 0) {
    const int sn = gp(w.sensor)[i];
    b |= (sn != 0 && sn != 1);
    if (!b) key = 2 * m + sn;
  }
  *bad = b;
  return key;
}

// A hit's input index (below 2^23: events hold at most 8,000,000 hits) and its
// key's position in its coarse bucket, packed into the fourth word of its
// coarse-order record.
__device__ __forceinline__ int hit_tag(int i, int key) { return i | ((key & (kFineKeys - 1)) << 23); }
__device__ __forceinline__ int tag_index(float t) { return __float_as_int(t) & 0x7fffff; }
__device__ __forceinline__ int tag_fine(float t) { return (int)((unsigned)__float_as_int(t) >> 23); }
static_assert(kFineBits + 23 <= 32, "index and fine key in one word");

// Lanes (of the active ones) whose `nbits`-bit value v equals this lane's.
__device__ __forceinline__ unsigned long long match_value(int v, int nbits, bool active) {
  unsigned long long m = __ballot(active);
  for (int b = 0; b < nbits; ++b) {
    const bool bit = (v >> b) & 1;
    const unsigned long long bb = __ballot(active && bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

__device__ __forceinline__ int bits_for(int n) {  // bits of the values 0 .. n - 1
  int b = 0;
  while ((1 << b) < n) ++b;
  return b;
}

// One block per tile of kHitTile hits, each of its four waves counting 1024
// consecutive hits into its own LDS row; the tile's coarse counts are the rows'
// sums (k_hits_scatter recounts the rows to rank its waves).
static_assert(kHitTile == kWaves * 1024, "a wave's part of a tile is 1024 hits");
__device__ __forceinline__ bool wave_coarse_counts(const Ws &w, int tb, int n_mod, int *row) {
  const int lane = lane_id(), wv = wave_id();
  bool any_bad = false;
  const int i0 = tb * kHitTile + wv * 1024, i1 = min(w.n_hits, i0 + 1024);
  for (int i = i0 + lane; i < i1; i += 64) {
    bool bad;
    const int key = hit_key(w, i, n_mod, &bad);
    any_bad |= bad;
    if (key >= 0) atomicAdd(&row[key >> kFineBits], 1);  // LDS
  }
  return any_bad;
}

// The four waves' rows of coarse counts live in dynamic LDS (kWaves x nc ints,
// sized at launch from the geometry), so small geometries keep more blocks
// resident.
__global__ __launch_bounds__(kBlock) void k_hits_count(const Ws *__restrict__ wb, int n_mod) {
  extern __shared__ int s_rows[];
  const Ws &w = wb[blockIdx.y];
  const int wv = wave_id();
  const int nc = n_coarse(n_mod), ntb = n_hit_tiles(w.n_hits);
  const int tb = blockIdx.x;
  if (tb < ntb) {
    for (int c = threadIdx.x; c < kWaves * nc; c += blockDim.x) s_rows[c] = 0;
    __syncthreads();
    if (wave_coarse_counts(w, tb, n_mod, s_rows + wv * nc)) atomicOr(&w.ctr[C_STATUS], (int)ST_BAD_HIT);
    __syncthreads();
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      int t = 0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q) t += s_rows[q * nc + c];
      gp(w.tile_hist)[(long)c * ntb + tb] = t;
    }
  }
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < w.n_seeds; s += gridDim.x * blockDim.x) {
    bool bad = !(w.q[s] == 1 || gp(w.q)[s] == -1) || !(isfinite(w.px[s]) && isfinite(w.py[s]) && isfinite(w.pz[s]));
    bad |= !(w.px[s] * gp(w.px)[s] + gp(w.py)[s] * gp(w.py)[s] > 0.0f);
    for (int k = 0; k < 4; ++k) {
      const int h = gp(w.hits4)[4 * s + k];
      bad |= (h < 0 || h >= w.n_hits);
      if (h >= 0 && h < w.n_hits) bad |= (w.module[h] != -1);
    }
    if (bad) atomicOr(&w.ctr[C_STATUS], (int)ST_BAD_SEED);
  }
}

// Stable scatter of a tile's hits into coarse-bucket order: each wave's first
// slot in bucket c is the tile's offset (the scan of the tile counts) plus the
// rows of the waves before it; in each round of 64 hits, a hit's rank among
// the round's hits of its bucket (match_value) places it.  The hit's
// coordinates, input index and key within its bucket travel with it (one
// 16-byte store), so the per-bucket sort reads them contiguously.
__global__ __launch_bounds__(kBlock) void k_hits_scatter(const Ws *__restrict__ wb, int n_mod) {
  extern __shared__ int s_rows[];  // kWaves x nc, as in k_hits_count
  const Ws &w = wb[blockIdx.y];
  const int wv = wave_id(), lane = lane_id();
  const int nc = n_coarse(n_mod), ntb = n_hit_tiles(w.n_hits);
  const int tb = blockIdx.x;
  if (tb >= ntb) return;  // the whole block
  for (int c = threadIdx.x; c < kWaves * nc; c += blockDim.x) s_rows[c] = 0;
  __syncthreads();
  (void)wave_coarse_counts(w, tb, n_mod, s_rows + wv * nc);
  __syncthreads();
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    int run = gp(w.tile_off)[(long)c * ntb + tb];
#pragma unroll
    for (int q = 0; q < kWaves; ++q) {
      const int v = s_rows[q * nc + c];
      s_rows[q * nc + c] = run;
      run += v;
    }
  }
  __syncthreads();
  int *s_run = s_rows + wv * nc;
  const int nbits = bits_for(nc);
  const int i0 = tb * kHitTile + wv * 1024, i1 = min(w.n_hits, i0 + 1024);
  for (int r0 = i0; r0 < i1; r0 += 64) {
    const int i = r0 + lane;
    bool bad = true;
    const int key = i < i1 ? hit_key(w, i, n_mod, &bad) : -1;
    const bool act = key >= 0;
    const int c = act ? key >> kFineBits : 0;
    const unsigned long long peers = match_value(c, nbits, act);
    int base = 0;
    if (act) {
      base = s_run[c];
      const int pos = base + lanes_below(peers);
      gstore(w.hcp, pos, make_float4(gp(w.x)[i], gp(w.y)[i], gp(w.z)[i], __int_as_float(hit_tag(i, key))));
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (act && lanes_below(peers) == 0) s_run[c] = base + __popcll(peers);  // the bucket's first lane
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// One block of kSortWaves waves per coarse bucket: the bucket's hits (in input
// order) are split into kSortWaves consecutive runs; each wave counts its
// run's keys, the block turns the counts into each (wave, key)'s first
// position (key order, then wave order: stable), writes the keys' offsets, and
// every wave places its run's hits 64 at a time in order.
constexpr int kSortWaves = 8;
__global__ __launch_bounds__(64 * kSortWaves) void k_bucket_sort(const Ws *__restrict__ wb, int n_mod) {
  __shared__ int s_cnt[kSortWaves][kFineKeys];
  __shared__ int s_key0[kFineKeys];
  const Ws &w = wb[blockIdx.y];
  const int wv = wave_id(), lane = lane_id(), t = threadIdx.x;
  const int nc = n_coarse(n_mod), ntb = n_hit_tiles(w.n_hits), nkeys = 2 * n_mod;
  const int c = blockIdx.x;
  if (c >= nc) return;  // the whole block
  const int j0 = gp(w.tile_off)[(long)c * ntb], j1 = gp(w.tile_off)[(long)(c + 1) * ntb];
  const long L = j1 - j0;
  const int a = j0 + (int)(L * wv / kSortWaves), b = j0 + (int)(L * (wv + 1) / kSortWaves);
  for (int f = lane; f < kFineKeys; f += 64) s_cnt[wv][f] = 0;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int j = a + lane; j < b; j += 64) atomicAdd(&s_cnt[wv][tag_fine(gload(w.hcp, j).w)], 1);  // LDS
  __syncthreads();
  // each key's total over the waves, then the keys' first positions (wave 0: one key per lane)
  int tot = 0;
  if (t < kFineKeys)
    for (int q = 0; q < kSortWaves; ++q) tot += s_cnt[q][t];
  if (t < kFineKeys) s_key0[t] = tot;
  __syncthreads();
  if (wv == 0) {
    static_assert(kFineKeys <= 64, "one key per lane");
    const int x0 = lane < kFineKeys ? s_key0[lane] : 0;
    int x = x0;
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    const int ex = j0 + x - x0;
    const int k = c * kFineKeys + lane;
    if (lane < kFineKeys) {
      s_key0[lane] = ex;
      if (k < nkeys) gp(w.boff)[k] = ex;
    }
    if (c == nc - 1 && lane == 0) gp(w.boff)[nkeys] = j1;
  }
  __syncthreads();
  // first position of each (wave, key): the key's first position plus the earlier waves' counts
  if (t < kFineKeys) {
    int run = s_key0[t];
    for (int q = 0; q < kSortWaves; ++q) {
      const int v = s_cnt[q][t];
      s_cnt[q][t] = run;
      run += v;
    }
  }
  __syncthreads();
  for (int r0 = a; r0 < b; r0 += 64) {
    const int j = r0 + lane;
    const bool act = j < b;
    const float4 h = act ? gload(w.hcp, j) : make_float4(0.f, 0.f, 0.f, 0.f);
    const int f = act ? tag_fine(h.w) : 0;
    const unsigned long long peers = match_value(f, kFineBits, act);
    int base = 0;
    if (act) {
      base = s_cnt[wv][f];
      const int pos = base + lanes_below(peers);
      gp(w.hidx)[pos] = tag_index(h.w);
      gstore(w.hpos, pos, make_float4(h.x, h.y, h.z, sqrtf(h.x * h.x + h.y * h.y)));
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (act && lanes_below(peers) == 0) s_cnt[wv][f] = base + __popcll(peers);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// ------------------------------------------------------------- a1: MD
constexpr int kMdStage = 128;  // hits per sensor staged in LDS per wave (more: read from HBM)
// MD stubs are stored as float2 or, with the geometry's 16-bit stub switch, as
// a dense array of binary16 pairs (rounded to nearest even) read back as float.
__device__ __forceinline__ void put_stub(const Ws &w, const DevGeom &g, int pos, float2 st) {
  if (g.stub16)
    gstore(reinterpret_cast<__half2 *>(w.md_stub), pos, __floats2half2_rn(st.x, st.y));
  else
    gstore(w.md_stub, pos, st);
}
__device__ __forceinline__ float2 get_stub(const Ws &w, const DevGeom &g, int i) {
  if (g.stub16) return __half22float2(gload(reinterpret_cast<const __half2 *>(w.md_stub), i));
  return gload(w.md_stub, i);
}

constexpr long kMdBig = 2048;  // modules with more pairs go to a whole block (k_md_big)
constexpr int kMdStageBig = 512;

// Anchor disc of a module for the segment stage's module-level azimuth
// pre-test, from the lower hits' bounding box (min/max reduced by the caller).
__device__ __forceinline__ float4 anchor_disc(float x0, float x1, float y0, float y1) {
  const float cx = 0.5f * (x0 + x1), cy = 0.5f * (y0 + y1);
  const float hx = 0.5f * (x1 - x0), hy = 0.5f * (y1 - y0);
  const float rho = sqrtf(hx * hx + hy * hy) * 1.0001f + 1e-3f;
  return make_float4(cx, cy, rho, sqrtf(cx * cx + cy * cy));
}

// Quotient and remainder of t / n for 0 <= t < 2^22 and n >= 1 from rn, the
// float reciprocal of n: t is exact in float and the two roundings (of 1 / n
// and of the product) are 2^-24 relative each, so the float quotient is within
// (t / n) 2^-23 < 1/2 of t / n; truncated, it is the quotient or one off, and
// one correction step each way makes it exact.  (Integer division has no
// instruction: the compiler's sequence for a variable divisor costs some 30
// instructions, in 64 bits far more.)
__device__ __forceinline__ int2 divmod22(int t, int n, float rn) {
  int q = (int)((float)t * rn);
  int r = t - q * n;
  if (r < 0) {
    --q;
    r += n;
  }
  if (r >= n) {
    ++q;
    r -= n;
  }
  return make_int2(q, r);
}

// One wave per module of at most kMdBig pairs; pairs (lower i, upper j) in
// row-major order, 64 at a time, compacted in order by ballot.  The fill also
// writes the module's anchor disc.
template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_md(const Ws *__restrict__ wb, DevGeom g) {
  const Ws &w = wb[blockIdx.y];
  __shared__ float4 s_lo[kWaves][kMdStage], s_up[kWaves][kMdStage];
  const int wv = wave_id(), lane = lane_id();
  const int wpb = blockDim.x >> 6;
  for (int m = blockIdx.x * wpb + wv; m < g.n_mod; m += gridDim.x * wpb) {
    const int lo0 = gp(w.boff)[2 * m], nlo = gp(w.boff)[2 * m + 1] - lo0;
    const int up0 = gp(w.boff)[2 * m + 1], nup = gp(w.boff)[2 * m + 2] - up0;
    const long npair = (long)nlo * nup;
    if (npair > kMdBig) {  // k_md_big's, listed for it (the list's order does not matter)
      if (!FILL && lane == 0) gp(w.md_dense)[atomicAdd(w.ctr + C_NDENSE, 1)] = m;
      continue;
    }
    if (npair == 0) {
      if (!FILL && lane == 0) gp(w.md_cnt)[m] = 0;
      continue;
    }
    for (int k = lane; k < nlo && k < kMdStage; k += 64) s_lo[wv][k] = gload(w.hpos, lo0 + k);
    for (int k = lane; k < nup && k < kMdStage; k += 64) s_up[wv][k] = gload(w.hpos, up0 + k);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const float4 win = gload(g.win, m);
    const ModInfo mi{gp(g.info)[m]};
    int base = FILL ? gp(w.md_off)[m] : 0;
    const int np = (int)npair;  // <= kMdBig here
    const float rnup = 1.0f / (float)nup;
    const int n_md = FILL ? gp(w.md_off)[m + 1] - base : 0;
    auto cache = gp(w.md_cache) + (long)kMdCache * m;
    const int md_keep = g.tiles.md_cache;
    if (FILL && n_md <= md_keep) {
      // the count pass kept this module's passing pairs (row-major order): copy them
      if (lane < n_md) {
        const int pk = cache[lane];
        const int i = pk >> 16, j = pk & 0xffff;
        const int pos = base + lane;
        if (pos < w.cap_md) {
          const float4 hi = i < kMdStage ? s_lo[wv][i] : gload(w.hpos, lo0 + i);
          const float4 hj = j < kMdStage ? s_up[wv][j] : gload(w.hpos, up0 + j);
          gstore(w.md_hits, pos, make_int2(gp(w.hidx)[lo0 + i], gp(w.hidx)[up0 + j]));
          gp(w.md_mod)[pos] = m;
          gstore(w.md_pos, pos, hi);
          put_stub(w, g, pos, md_stub(hi, hj, mi));
        }
      }
    }
    for (int p0 = 0; p0 < np && !(FILL && n_md <= md_keep); p0 += 64) {
      const int p = p0 + lane;
      bool pass = false;
      int i = 0, j = 0;
      float4 hi, hj;
      if (p < np) {
        const int2 ij = divmod22(p, nup, rnup);
        i = ij.x;
        j = ij.y;
        hi = i < kMdStage ? s_lo[wv][i] : gload(w.hpos, lo0 + i);
        hj = j < kMdStage ? s_up[wv][j] : gload(w.hpos, up0 + j);
        pass = md_pass(hi, hj, win, mi);
      }
      const unsigned long long bm = __ballot(pass);
      if (FILL && pass) {
        const int pos = base + lanes_below(bm);
        if (pos < w.cap_md) {
          gstore(w.md_hits, pos, make_int2(gp(w.hidx)[lo0 + i], gp(w.hidx)[up0 + j]));
          gp(w.md_mod)[pos] = m;
          gstore(w.md_pos, pos, hi);
          put_stub(w, g, pos, md_stub(hi, hj, mi));
        }
      }
      if (!FILL && pass) {
        const int r = base + lanes_below(bm);
        if (r < md_keep) cache[r] = (i << 16) | j;
      }
      base += __popcll(bm);
    }
    if (!FILL) {
      if (lane == 0) gp(w.md_cnt)[m] = base;
    } else {
      // a disc in x-y around every anchor of this module (the lower hits' bounding box)
      float x0 = 3.0e38f, x1 = -3.0e38f, y0 = 3.0e38f, y1 = -3.0e38f;
      for (int k = lane; k < nlo; k += 64) {
        const float4 h = k < kMdStage ? s_lo[wv][k] : gload(w.hpos, lo0 + k);
        x0 = fminf(x0, h.x); x1 = fmaxf(x1, h.x);
        y0 = fminf(y0, h.y); y1 = fmaxf(y1, h.y);
      }
      for (int o = 32; o > 0; o >>= 1) {
        x0 = fminf(x0, __shfl_xor(x0, o, 64)); x1 = fmaxf(x1, __shfl_xor(x1, o, 64));
        y0 = fminf(y0, __shfl_xor(y0, o, 64)); y1 = fmaxf(y1, __shfl_xor(y1, o, 64));
      }
      if (lane == 0) gstore(w.mod_disc, m, anchor_disc(x0, x1, y0, y1));
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// The same for the modules with more than kMdBig pairs (listed by the count
// pass of k_md), one block (kBlock threads) each, so that no single wave
// carries a dense module and no block walks the modules that are not dense: the block
// (one wave per part: `parts` = blockDim.x / 64 <= kMdParts) stages both
// sensors' hits, and each of its waves takes one consecutive part of the
// module's row-major pairs on its own (no block barrier per round).  Sixteen
// parts keep the densest module (~24,000 pairs on PU200) from setting the
// kernel's end when a launch holds one event; over many events four parts
// run faster.  The count pass writes each part's count (md_part), from which
// the fill starts each part at the module's offset plus the counts of the
// parts before it, so the module's MDs stay in row-major order; it also keeps
// each part's first kMdParts * kMdQCache / parts passing pairs, so the fill of
// a part with no more than that copies them instead of testing every pair
// again.
template <bool FILL>
__global__ __launch_bounds__(64 * kMdParts) void k_md_big(const Ws *__restrict__ wb, DevGeom g) {
  const Ws &w = wb[blockIdx.y];
  __shared__ float4 s_lo[kMdStageBig], s_up[kMdStageBig];
  __shared__ int s_part[kMdParts];
  __shared__ float4 s_box[kMdParts];
  const int parts = blockDim.x >> 6, qcap = kMdParts * kMdQCache / parts;
  const int wid = wave_id(), lane = lane_id();
  const int n_dense = uload(w.ctr + C_NDENSE);
  for (int kd = blockIdx.x; kd < n_dense; kd += gridDim.x) {
    const int m = uload(w.md_dense + kd);
    const int lo0 = gp(w.boff)[2 * m], nlo = gp(w.boff)[2 * m + 1] - lo0;
    const int up0 = gp(w.boff)[2 * m + 1], nup = gp(w.boff)[2 * m + 2] - up0;
    const long npair = (long)nlo * nup;
    if (npair <= kMdBig) continue;
    __syncthreads();  // the previous module's LDS reads are done
    for (int k = threadIdx.x; k < nlo && k < kMdStageBig; k += blockDim.x) s_lo[k] = gload(w.hpos, lo0 + k);
    for (int k = threadIdx.x; k < nup && k < kMdStageBig; k += blockDim.x) s_up[k] = gload(w.hpos, up0 + k);
    __syncthreads();
    const float4 win = gload(g.win, m);
    const ModInfo mi{gp(g.info)[m]};
    const float rnup = 1.0f / (float)nup;
    const bool small = npair < (1L << 22);  // divmod22's range (always, below 2,048 hits per sensor)
    const long q0 = npair * wid / parts, q1 = npair * (wid + 1) / parts;  // this wave's part
    // the count pass keeps a part's first qcap passing pairs (indices < 2^16)
    const bool packable = nlo <= 0xffff && nup <= 0xffff;
    unsigned *qcache = reinterpret_cast<unsigned *>(w.md_bcache) + (long)m * kMdParts * kMdQCache + wid * qcap;
    int base = 0, qn = 0;
    if (FILL) {
      base = gp(w.md_off)[m];
      for (int q = 0; q < wid; ++q) base += gp(w.md_part)[(long)kMdParts * m + q];
      qn = gp(w.md_part)[(long)kMdParts * m + wid];
    }
    const bool cached = FILL && packable && qn <= qcap;
    if (cached) {  // the part's MDs from the count pass's pairs, in the same order
      for (int k = lane; k < qn; k += 64) {
        const unsigned e = gp(qcache)[k];
        const int i = (int)(e >> 16), j = (int)(e & 0xffffu);
        const float4 hi = i < kMdStageBig ? s_lo[i] : gload(w.hpos, lo0 + i);
        const float4 hj = j < kMdStageBig ? s_up[j] : gload(w.hpos, up0 + j);
        const int pos = base + k;
        if (pos < w.cap_md) {
          gstore(w.md_hits, pos, make_int2(gp(w.hidx)[lo0 + i], gp(w.hidx)[up0 + j]));
          gp(w.md_mod)[pos] = m;
          gstore(w.md_pos, pos, hi);
          put_stub(w, g, pos, md_stub(hi, hj, mi));
        }
      }
    }
    for (long p0 = q0; p0 < (cached ? q0 : q1); p0 += 64) {
      const long p = p0 + lane;
      bool pass = false;
      int i = 0, j = 0;
      float4 hi, hj;
      if (p < q1) {
        if (small) {
          const int2 ij = divmod22((int)p, nup, rnup);
          i = ij.x;
          j = ij.y;
        } else {
          i = (int)(p / nup);
          j = (int)(p - (long)i * nup);
        }
        hi = i < kMdStageBig ? s_lo[i] : gload(w.hpos, lo0 + i);
        hj = j < kMdStageBig ? s_up[j] : gload(w.hpos, up0 + j);
        pass = md_pass(hi, hj, win, mi);
      }
      const unsigned long long bm = __ballot(pass);
      if (!FILL && pass && packable) {
        const int r = base + lanes_below(bm);
        if (r < qcap) gp(qcache)[r] = ((unsigned)i << 16) | (unsigned)j;
      }
      if (FILL && pass) {
        const int pos = base + lanes_below(bm);
        if (pos < w.cap_md) {
          gstore(w.md_hits, pos, make_int2(gp(w.hidx)[lo0 + i], gp(w.hidx)[up0 + j]));
          gp(w.md_mod)[pos] = m;
          gstore(w.md_pos, pos, hi);
          put_stub(w, g, pos, md_stub(hi, hj, mi));
        }
      }
      base += __popcll(bm);
    }
    if (!FILL) {
      if (lane == 0) {
        gp(w.md_part)[(long)kMdParts * m + wid] = base;
        s_part[wid] = base;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        int c = 0;
        for (int q = 0; q < parts; ++q) c += s_part[q];
        gp(w.md_cnt)[m] = c;
      }
    } else {
      float x0 = 3.0e38f, x1 = -3.0e38f, y0 = 3.0e38f, y1 = -3.0e38f;
      for (int k = threadIdx.x; k < nlo; k += blockDim.x) {
        const float4 h = k < kMdStageBig ? s_lo[k] : gload(w.hpos, lo0 + k);
        x0 = fminf(x0, h.x); x1 = fmaxf(x1, h.x);
        y0 = fminf(y0, h.y); y1 = fmaxf(y1, h.y);
      }
      for (int o = 32; o > 0; o >>= 1) {
        x0 = fminf(x0, __shfl_xor(x0, o, 64)); x1 = fmaxf(x1, __shfl_xor(x1, o, 64));
        y0 = fminf(y0, __shfl_xor(y0, o, 64)); y1 = fmaxf(y1, __shfl_xor(y1, o, 64));
      }
      if (lane == 0) s_box[wid] = make_float4(x0, x1, y0, y1);
      __syncthreads();
      if (threadIdx.x == 0) {
        for (int q = 1; q < parts; ++q) {
          x0 = fminf(x0, s_box[q].x); x1 = fmaxf(x1, s_box[q].y);
          y0 = fminf(y0, s_box[q].z); y1 = fmaxf(y1, s_box[q].w);
        }
        gstore(w.mod_disc, m, anchor_disc(x0, x1, y0, y1));
      }
    }
  }
}

// ------------------------------------------------------------- a2: LS
// Pre-tests of the segment azimuth window that only save work.  For inner
// anchor A and a partner module whose anchors lie in an x-y disc (centre C,
// radius rho; written by the MD fill), every term of ls_pass's window W is at
// most its value at the largest partner radius r_B <= |C| + rho: the
// threshold term (ub - ua) / sqrt(1 - ub^2) and the impact-parameter term
// D0 (1/r_A - 1/r_B) grow with r_B (the latter is below D0 / r_A) and the
// pitch terms are below (h_A + h_B) / r_A for an outgoing segment.  With the
// margins below (far above rounding) Wmax >= W, so a candidate failing
// |A x B| <= Wmax r_A r_B fails ls_pass; and since |A x B| = r_A |n.B| >= r_A
// (|n.C| - rho) for the unit normal n of A, with r_B <= |C| + rho, a module
// failing |n.C| - rho <= Wmax (|C| + rho) has no candidate that can pass.
//
// The pre-tests use the hardware reciprocal, reciprocal square root and
// square root (v_rcp_f32, v_rsq_f32, v_sqrt_f32: within 1 ulp each) instead of
// correctly rounded division and square root; their results differ from the
// exact values by a few parts in 1e7, far inside each pre-test's margin, so
// the pre-tests stay supersets of the exact selection that decides.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }

__device__ __forceinline__ float ls_window_bound(const float4 &A, ModInfo ma, float4 disc, ModInfo mb, float d0) {
  const float ub = kHalfKmax * ((disc.w + disc.z) + mb.er());
  if (!(ub < 0.99f)) return 3.0e38f;  // no useful bound
  const float ua = kHalfKmax * (A.w - ma.er());
  const float w = (ub - ua) * frsq(1.0f - ub * ub) + (d0 + ma.hphi() + 0.005f) * frcp(A.w);
  return (w * kMargin + kEps) * 1.01f + 1e-6f;
}

__device__ __forceinline__ bool ls_module_may_pass(const float4 &A, float4 disc, float wmax) {
  const float dn = fabsf(A.x * disc.y - A.y * disc.x) * frcp(A.w);
  return dn - disc.z <= (wmax * (disc.w + disc.z)) * 1.001f + 1e-4f;
}

// One MD's stub check of ls_pass (ls_stub_ok) evaluated with the fast
// operations, from the chord (sx, sy) = B - A, its inverse length il, dz = zB -
// zA, the chord's sine sn against the radial direction the check uses, eang
// and the MD's radius rp: every quantity is within 2e-6 relative of the exact
// one (a chain of at most six operations of <= 2 ulp), except that 1 - s^2
// loses relative precision as s^2 -> 1: chords within asin(sqrt(0.9)) of the
// tangent skip the pre-test (the exact test decides), which bounds the error of
// the predicted displacement at 4e-5 relative.  The margins (1e-4 of the
// prediction and of the error) exceed those bounds, so whatever passes the
// exact check passes this one.
__device__ __forceinline__ bool ls_stub_may_pass(float2 st, ModInfo m, float sn, float sx, float sy, float il, float dz,
                                                 float eang, float rp, float d0) {
  float pred, err;
  if (!m.endcap()) {
    const float sn2 = sn * sn;
    if (!(sn2 < 0.9f)) return true;
    pred = (st.y * sn) * frsq(1.0f - sn2);
    err = 2.0f * m.hphi() + (2.0f * st.y) * (eang + d0 * frcp(rp));
  } else {
    const float adz = fabsf(dz);
    if (!(adz > 0.0f)) return false;  // the exact check's own rejection, on the same operands
    const float ds = st.y * (sx * sx + sy * sy) * il * frcp(adz);
    pred = ds * sn;
    err = (2.0f * m.hphi() + (float)0.03 * fabsf(pred)) + ds * (eang + d0 * frcp(rp));
  }
  return fabsf(st.x - pred) <= (err * kMargin) * 1.0001f + kEps + 1e-4f * fabsf(pred);
}

// The inner MD's stub check (its chord sine taken at the outer anchor B).
__device__ __forceinline__ bool ls_inner_stub_may_pass(const float4 &A, const float4 &B, float2 st, ModInfo ma,
                                                       ModInfo mb, float d0) {
  const float sx = B.x - A.x, sy = B.y - A.y;
  const float il = frsq(sx * sx + sy * sy);  // 1 / |AB|
  const float sn = (B.x * sy - B.y * sx) * frcp(B.w) * il;
  const float ea2 = ma.endcap() ? ma.hlong() : ma.hphi();
  const float eb2 = mb.endcap() ? mb.hlong() : mb.hphi();
  return ls_stub_may_pass(st, ma, sn, sx, sy, il, B.z - A.z, (ea2 + eb2) * il, A.w, d0);
}

__device__ __forceinline__ bool ls_window_may_pass(const float4 &A, const float4 &B, float wmax) {
  const float c = A.x * B.y - A.y * B.x;
  return fabsf(c) <= wmax * (A.w * B.w);
}

// The checks of ls_pass that a pair past the two pre-tests above still fails
// most often, on the pair itself: the signs of dr and of A.B (the same
// operations as ls_pass), the x-y window with the outer radius of this B
// instead of the module's (all terms of w are positive for dr > 0, so the fast
// operations' few-ulp errors stay far inside the 1e-4 margin; ub >= 0.99
// leaves the decision to the exact test), and the outer MD's stub check, its
// chord sine taken at the inner anchor A.
__device__ __forceinline__ bool ls_pair_may_pass(const float4 &A, const float4 &B, float2 sb, ModInfo ma, ModInfo mb,
                                                 float d0) {
  const float dr = B.w - A.w;
  if (!(dr > 0.0f)) return false;
  if (!(A.x * B.x + A.y * B.y > 0.0f)) return false;
  const float ub = kHalfKmax * (B.w + mb.er());
  if (ub < 0.99f) {
    const float ua = kHalfKmax * (A.w - ma.er());
    const float ra = frcp(A.w), rb = frcp(B.w);
    const float wv = (ub - ua) * frsq(1.0f - ub * ub) + (d0 * dr) * (ra * rb) + ma.hphi() * ra + mb.hphi() * rb;
    const float c = A.x * B.y - A.y * B.x;
    if (!(fabsf(c) <= ((wv * kMargin + kEps) * (A.w * B.w)) * 1.0001f + 1e-6f)) return false;
  }
  const float sx = B.x - A.x, sy = B.y - A.y;
  const float il = frsq(sx * sx + sy * sy);
  const float sn = (A.x * sy - A.y * sx) * frcp(A.w) * il;
  const float ea2 = ma.endcap() ? ma.hlong() : ma.hphi();
  const float eb2 = mb.endcap() ? mb.hlong() : mb.hphi();
  return ls_stub_may_pass(sb, mb, sn, sx, sy, il, B.z - A.z, (ea2 + eb2) * il, B.w, d0);
}

constexpr int kMaxEdges = 128;  // module-map targets per module (checked when the geometry is loaded)

// Drops the first 64 entries of a wave's queue (two arrays of 128): the rest (< 64)
// entries behind them move to its front.
template <class T>
__device__ __forceinline__ void queue_pop64(int *qa, T *qb, int rest) {
  const int lane = lane_id();
  int va = 0;
  T vb = 0;
  if (lane < rest) {
    va = qa[64 + lane];
    vb = qb[64 + lane];
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (lane < rest) {
    qa[lane] = va;
    qb[lane] = vb;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void queue_pop64(int *qa, int rest) {
  const int lane = lane_id();
  const int va = lane < rest ? qa[64 + lane] : 0;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (lane < rest) qa[lane] = va;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Fill pass of the segment search for the inner MDs with more segments than
// the count pass cached (k_ls_copy writes the others and lists these densely):
// one wave per inner MD a.  Its candidates -- the MDs of every module linked
// to a's module, edge by edge -- are flattened into one list that the 64
// lanes stride over, so a wave stays full even though each linked module
// holds few MDs; candidates past the pre-tests, then past the pair pre-test,
// are compacted in list order with ballot and mbcnt into two LDS queues, and
// the full selection runs on full waves of the second.
// Eight waves per SIMD (64 VGPRs; a few spill): the segment search is bound by
// the latency of its dependent gathers, and more resident waves hide more of
// it (measured 9% faster than the 77-VGPR, six-wave build; the same for the
// triplet and quintuplet searches made them slower).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_ls_fill(const Ws *__restrict__ wb,
                                                                                             DevGeom g) {
  const Ws &w = wb[blockIdx.y];
  __shared__ int s_pre[kWaves][kMaxEdges + 1];  // running MD count before each edge
  __shared__ int s_first[kWaves][kMaxEdges];    // first MD of each linked module
  __shared__ int s_info[kWaves][kMaxEdges];
  __shared__ float s_wmax[kWaves][kMaxEdges];   // window bound of each linked module
  // candidates in order, as partner | module info << 30: past the candidate pre-tests
  // (s_q) and past the pair pre-test as well (s_r)
  __shared__ int s_q[kWaves][128], s_r[kWaves][128];
  const int n_md = uload(w.ctr + C_NMD);
  const int wv = wave_id(), lane = lane_id();
  const int wpb = blockDim.x >> 6;  // waves per block (a tuned launch may run fewer than kWaves)
  const int waves_total = gridDim.x * wpb;
  auto process = [&](const int a) {
    const int ma = gp(w.md_mod)[a];
    const float4 A = gload(w.md_pos, a);
    const float2 sa = get_stub(w, g, a);
    const ModInfo mia{gp(g.info)[ma]};
    const int e0 = gp(g.map_off)[ma];
    const int ne = gp(g.map_off)[ma + 1] - e0;  // <= kMaxEdges, checked when the geometry is loaded
    // per-edge MD ranges and their exclusive prefix over the wave
    int run = 0;
    for (int k0 = 0; k0 < ne; k0 += 64) {
      const int k = k0 + lane;
      int first = 0, cnt = 0, info = 0;
      float wm = 0.0f;
      if (k < ne) {
        const int mb = gp(g.map_tgt)[e0 + k];
        first = gp(w.md_off)[mb];
        const int last = min(w.md_off[mb + 1], n_md);
        cnt = last > first ? last - first : 0;
        info = gp(g.info)[mb];
        if (cnt > 0) {
          const float4 disc = gload(w.mod_disc, mb);
          wm = ls_window_bound(A, mia, disc, ModInfo{info}, g.d0max);
          if (!ls_module_may_pass(A, disc, wm)) cnt = 0;
        }
      }
      int x = cnt;
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      if (k < ne) {
        s_pre[wv][k] = run + x - cnt;
        s_first[wv][k] = first;
        s_info[wv][k] = info;
        s_wmax[wv][k] = wm;
      }
      run += __shfl(x, 63, 64);
    }
    if (lane == 0) s_pre[wv][ne] = run;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int total = run;
    int out = gp(w.ls_off)[a];
    // the pair pre-test on the first n candidates of s_q (n <= 64); the passing ones join s_r
    int nr = 0;
    auto sift = [&](int n) {
      bool ok = false;
      int e = 0;
      if (lane < n) {
        e = s_q[wv][lane];
        const int b = e & 0x3fffffff;
        ok = ls_pair_may_pass(A, gload(w.md_pos, b), get_stub(w, g, b), mia, ModInfo{(int)((unsigned)e >> 30)},
                              g.d0max);
      }
      const unsigned long long m = __ballot(ok);
      if (ok) s_r[wv][nr + lanes_below(m)] = e;
      nr += __popcll(m);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    };
    // the full selection on the first n candidates of s_r (n <= 64), in candidate order
    auto select = [&](int n) {
      bool pass = false;
      int b = 0, info = 0;
      float2 beta = make_float2(0.f, 0.f);
      if (lane < n) {
        const int e = s_r[wv][lane];
        b = e & 0x3fffffff;
        info = (int)((unsigned)e >> 30);
        pass = ls_pass(A, gload(w.md_pos, b), sa, get_stub(w, g, b), mia, ModInfo{info}, &beta, g.d0max);
      }
      const unsigned long long m = __ballot(pass);
      const int pre = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
      const int pos = out + pre;
      if (pass && pos < w.cap_ls) {
        gstore(w.ls_md, pos, make_int2(a, b));
        gstore(w.ls_beta, pos, beta);
        gstore(w.ls_opos, pos, gload(w.md_pos, b));
        gp(w.ls_oinf)[pos] = info;
      }
      out += __popcll(m);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    };
    // candidates past the azimuth pre-tests and the inner MD's own stub check (both
    // necessary conditions of ls_pass) are queued in LDS, and the full selection runs
    // on full waves of them
    int nq = 0;
    int e = 0;  // edge of this lane's candidate (candidates advance monotonically)
    for (int c0 = 0; c0 < total; c0 += 64) {
      const int c = c0 + lane;
      bool keep = false;
      int b = 0, info = 0;
      if (c < total) {
        while (s_pre[wv][e + 1] <= c) ++e;
        b = s_first[wv][e] + (c - s_pre[wv][e]);
        const float4 Bp = gload(w.md_pos, b);
        info = s_info[wv][e];
        keep = ls_window_may_pass(A, Bp, s_wmax[wv][e]) &&
               ls_inner_stub_may_pass(A, Bp, sa, mia, ModInfo{info}, g.d0max);
      }
      const unsigned long long m = __ballot(keep);
      const int pre = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
      if (keep) s_q[wv][nq + pre] = b | (info << 30);
      nq += __popcll(m);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // each queue holds < 64 entries before a round adds at most 64
      if (nq >= 64) {
        sift(64);
        queue_pop64(s_q[wv], nq - 64);
        nq -= 64;
        if (nr >= 64) {
          select(64);
          queue_pop64(s_r[wv], nr - 64);
          nr -= 64;
        }
      }
    }
    if (nq > 0) sift(nq);
    while (nr > 0) {
      const int n2 = nr < 64 ? nr : 64;
      select(n2);
      queue_pop64(s_r[wv], nr - n2);
      nr -= n2;
    }
  };
  const int n_ovf = uload(w.ctr + C_NLSOVF);
  for (int k = blockIdx.x * wpb + wv; k < n_ovf; k += waves_total) process(w.ls_ovf[k]);
}


// Count pass of the segment search: one wave per group of up to kLsGroup
// consecutive inner MDs, taken in chunks of MDs of one module whose (inner MD,
// linked module) pairs are flattened over the lanes.  Each candidate goes
// through the pre-tests as in k_ls_fill, but the queue of candidates past them
// is shared by the group.  Full waves of queued pairs then go through a second,
// pair-level pre-test (ls_pair_may_pass: about a third of them pass on PU200
// events), and its survivors, queued the same way, through the full selection,
// which thus runs on full waves of likely pairs rather than on the ~15 a single
// MD queues.  The pairs of one inner MD are consecutive in both queues; a
// passing pair's rank among its MD's passing pairs is the MD's count from
// earlier flushes plus the passing lanes of its run below it.  Writes each MD's count and caches up to tiles.ls_cache
// partners in candidate order.  The group size trades the fuller selection
// waves against the number of waves in flight (tiles.ls_group; see
// ls_group_for).
constexpr int kLsPairs = kMaxEdges;  // (inner MD, linked module) pairs of a chunk in LDS

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) void k_ls_count(
    const Ws *__restrict__ wb, DevGeom g, int group) {
  const Ws &w = wb[blockIdx.y];
  // (inner MD, linked module) pairs left with candidates, in (MD, map) order: first MD of
  // the linked module, candidates before it, module info, window bound (bits); and the
  // pair's inner MD (its slot in the group)
  __shared__ int4 s_edge[kWaves][kLsPairs];
  __shared__ int s_ek[kWaves][kLsPairs];
  __shared__ int s_mark[kWaves][64];            // a pair's candidates start here
  // (inner MD, candidate) pairs in order, as partner | module info << 30 and the inner
  // MD's slot in the group: past the candidate pre-tests (s_q) and past the pair
  // pre-test as well (s_r)
  __shared__ int s_q[kWaves][128], s_r[kWaves][128];
  __shared__ unsigned char s_qg[kWaves][128], s_rg[kWaves][128];
  __shared__ float4 s_A[kWaves][kLsGroup];      // the group's inner MDs
  __shared__ float2 s_sa[kWaves][kLsGroup];
  __shared__ int s_mia[kWaves][kLsGroup], s_cnt[kWaves][kLsGroup], s_mm[kWaves][kLsGroup];
  const int n_md = uload(w.ctr + C_NMD);
  const int wv = wave_id(), lane = lane_id();
  const int wpb = blockDim.x >> 6;
  const int waves_total = gridDim.x * wpb;
  const int n_grp = (n_md + group - 1) / group;
  const int keep = g.tiles.ls_cache;
  for (int gi = blockIdx.x * wpb + wv; gi < n_grp; gi += waves_total) {
    const int a0 = gi * group;
    const int na = min(group, n_md - a0);
    if (lane < na) {
      const int a = a0 + lane;
      const int ma = gp(w.md_mod)[a];
      s_A[wv][lane] = gload(w.md_pos, a);
      s_sa[wv][lane] = get_stub(w, g, a);
      s_mia[wv][lane] = gp(g.info)[ma];
      s_mm[wv][lane] = ma;
      s_cnt[wv][lane] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // the pair pre-test on the first n pairs of s_q (n <= 64); the passing ones join s_r
    int nr = 0;
    auto sift = [&](int n) {
      bool ok = false;
      int e = 0, q = 0;
      if (lane < n) {
        e = s_q[wv][lane];
        q = s_qg[wv][lane];
        const int b = e & 0x3fffffff;
        ok = ls_pair_may_pass(s_A[wv][q], gload(w.md_pos, b), get_stub(w, g, b), ModInfo{s_mia[wv][q]},
                              ModInfo{(int)((unsigned)e >> 30)}, g.d0max);
      }
      const unsigned long long m = __ballot(ok);
      if (ok) {
        const int pos = nr + lanes_below(m);
        s_r[wv][pos] = e;
        s_rg[wv][pos] = (unsigned char)q;
      }
      nr += __popcll(m);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    };
    // the full selection on the first n pairs of s_r (n <= 64)
    auto select = [&](int n) {
      bool pass = false;
      int e = 0, q = -1;
      if (lane < n) {
        e = s_r[wv][lane];
        q = s_rg[wv][lane];
        const int b = e & 0x3fffffff;
        float2 beta;
        pass = ls_pass(s_A[wv][q], gload(w.md_pos, b), s_sa[wv][q], get_stub(w, g, b), ModInfo{s_mia[wv][q]},
                       ModInfo{(int)((unsigned)e >> 30)}, &beta, g.d0max);
      }
      const unsigned long long m = __ballot(pass);
      const int qp = __shfl_up(q, 1, 64), qn = __shfl_down(q, 1, 64);
      const unsigned long long starts = __ballot(lane == 0 || q != qp);
      const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
      const int first = 63 - __clzll(starts & upto);  // first lane of this lane's run
      const int below = __popcll(m & ((1ull << lane) - 1ull) & ~((1ull << first) - 1ull));
      int before = 0;
      if (lane < n) before = s_cnt[wv][q];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (pass && before + below < keep)  // the partner and its module's info word (2 bits) in one int
        gp(w.ls_cache)[(long)(a0 + q) * kLsCache + before + below] = e;
      if (lane < n && (lane == n - 1 || qn != q)) s_cnt[wv][q] = before + below + (pass ? 1 : 0);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    };
    int nq = 0;
    // the linked modules' data of the current inner module (one per lane, when it has
    // at most 64 of them): consecutive inner MDs mostly share their module
    int cur_ma = -1, e0 = 0, ne = 0;
    int r_first = 0, r_cnt = 0, r_info = 0;
    float4 r_disc = make_float4(0.f, 0.f, 0.f, 0.f);
    auto linked = [&](int kk, int &first, int &cnt, int &info, float4 &disc) {
      const int mb = gp(g.map_tgt)[e0 + kk];
      first = gp(w.md_off)[mb];
      const int last = min(gp(w.md_off)[mb + 1], n_md);
      cnt = last > first ? last - first : 0;
      info = gp(g.info)[mb];
      disc = gload(w.mod_disc, mb);
    };
    // Chunks of consecutive inner MDs of one module, at most kLsPairs / ne of them, so
    // that every (inner MD, linked module) pair of the chunk fits the LDS list: the
    // prologue and the candidate rounds run over the chunk's pairs flattened, which
    // fills the lanes that one MD's ~27 linked modules and ~90 candidates leave idle.
    for (int k0 = 0; k0 < na;) {
      const int ma = __builtin_amdgcn_readfirstlane(s_mm[wv][k0]);
      if (ma != cur_ma) {
        cur_ma = ma;
        e0 = uload(g.map_off + ma);
        ne = uload(g.map_off + ma + 1) - e0;  // <= kMaxEdges = kLsPairs, checked when the geometry is loaded
        if (ne <= 64 && lane < ne) linked(lane, r_first, r_cnt, r_info, r_disc);
      }
      const int cap_k = ne > 0 ? kLsPairs / ne : na;
      int k1 = k0 + 1;
      while (k1 < na && k1 - k0 < cap_k && __builtin_amdgcn_readfirstlane(s_mm[wv][k1]) == ma) ++k1;
      const int npair = (k1 - k0) * ne;
      const float rne = ne > 0 ? 1.0f / (float)ne : 0.0f;
      int run = 0, n_ne = 0;
      for (int p0 = 0; p0 < npair; p0 += 64) {
        const int p = p0 + lane;
        const int2 ke = divmod22(p < npair ? p : 0, ne > 0 ? ne : 1, rne);  // (MD of the chunk, link)
        int first = 0, cnt = 0, info = 0;
        float4 disc = r_disc;
        if (ne <= 64) {  // the links' data from the lanes that hold them
          first = __shfl(r_first, ke.y, 64);
          cnt = __shfl(r_cnt, ke.y, 64);
          info = __shfl(r_info, ke.y, 64);
          disc = make_float4(__shfl(r_disc.x, ke.y, 64), __shfl(r_disc.y, ke.y, 64), __shfl(r_disc.z, ke.y, 64),
                             __shfl(r_disc.w, ke.y, 64));
        }
        float wm = 0.0f;
        const int kk = k0 + ke.x;
        if (p < npair) {
          if (ne > 64) linked(ke.y, first, cnt, info, disc);
          if (cnt > 0) {
            const float4 A = s_A[wv][kk];
            const ModInfo mia{s_mia[wv][kk]};
            wm = ls_window_bound(A, mia, disc, ModInfo{info}, g.d0max);
            if (!ls_module_may_pass(A, disc, wm)) cnt = 0;
          }
        } else {
          cnt = 0;
        }
        int x = cnt;
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(x, o, 64);
          if (lane >= o) x += y;
        }
        const unsigned long long live = __ballot(cnt > 0);
        if (cnt > 0) {
          const int q = n_ne + lanes_below(live);
          s_edge[wv][q] = make_int4(first, run + x - cnt, info, __float_as_int(wm));
          s_ek[wv][q] = kk;
        }
        n_ne += __popcll(live);
        run += __builtin_amdgcn_readfirstlane(__shfl(x, 63, 64));
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      const int total = run;
      // Candidates go 64 per round.  The candidate c of lane L lies in the last pair whose
      // candidates start at or before c: the pairs starting before the round (jlo of
      // them) plus those starting at or below L in it, found by marking the round's
      // starts (distinct, as every listed pair has candidates) and a ballot.
      int jlo = 0;
      // at least one round, so that the group's last chunk flushes the queue
      for (int c0 = 0; c0 < (total > 0 ? total : 1); c0 += 64) {
        s_mark[wv][lane] = 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (jlo + lane < n_ne) {
          const int p = s_edge[wv][jlo + lane].y - c0;  // >= 0: it starts at or after c0
          if (p < 64) s_mark[wv][p] = 1;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const unsigned long long starts = __ballot(s_mark[wv][lane] != 0);
        const int c = c0 + lane;
        bool keep_c = false;
        int b = 0, info = 0, kk = 0;
        if (c < total) {
          const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
          const int j = jlo - 1 + __popcll(starts & upto);
          const int4 E = s_edge[wv][j];
          kk = s_ek[wv][j];
          const float4 A = s_A[wv][kk];
          const float2 sa = s_sa[wv][kk];
          const ModInfo mia{s_mia[wv][kk]};
          b = E.x + (c - E.y);
          const float4 Bp = gload(w.md_pos, b);
          info = E.z;
          keep_c = ls_window_may_pass(A, Bp, __int_as_float(E.w)) &&
                   ls_inner_stub_may_pass(A, Bp, sa, mia, ModInfo{info}, g.d0max);
        }
        jlo += __popcll(starts);
        const unsigned long long m = __ballot(keep_c);
        if (keep_c) {
          const int pos = nq + lanes_below(m);
          s_q[wv][pos] = b | (info << 30);
          s_qg[wv][pos] = (unsigned char)kk;
        }
        nq += __popcll(m);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // each queue holds < 64 entries before a round adds at most 64, and is drained
        // 64 at a time; the group's last round drains both completely
        const bool fin = k1 == na && c0 + 64 >= total;
        while (nq >= 64 || (fin && nq > 0)) {
          const int n1 = nq < 64 ? nq : 64;
          sift(n1);
          queue_pop64(s_q[wv], s_qg[wv], nq - n1);
          nq -= n1;
          while (nr >= 64) {
            select(64);
            queue_pop64(s_r[wv], s_rg[wv], nr - 64);
            nr -= 64;
          }
        }
        if (fin && nr > 0) {
          select(nr);
          nr = 0;
        }
      }
      k0 = k1;
    }
    if (lane < na) {
      const int c = s_cnt[wv][lane];
      gp(w.ls_cnt)[a0 + lane] = c;
      gp(w.ls_ovf_flag)[a0 + lane] = c > keep ? 1 : 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// ---- flattened pair search shared by T3 and T5: a wave takes 64 consecutive
// parents (one per lane), stages what their pairs need in LDS, prefix-sums
// their candidate counts and lets its 64 lanes stride over all (parent,
// candidate) pairs in order, so a parent with many candidates does not hold
// the wave.  The rank of an accepted pair among its parent's accepted pairs
// (its output position after the parent's offset in the fill) is the
// parent's count from earlier rounds plus the accepted pairs of the same
// parent on lower lanes of this round (a parent's pairs are on consecutive
// lanes).  COUNT writes the per-parent counts, FILL the objects.
__device__ __forceinline__ int pair_rank(unsigned long long m, int seg_first_lane, int before_round) {
  return before_round + lanes_below(m) - __popcll(m & ((1ull << seg_first_lane) - 1ull));
}
// Exclusive prefix of n over the wave into seg[0..64] (seg[64] = total); returns the total.
__device__ __forceinline__ int wave_segments(int n, int *seg) {
  const int lane = lane_id();
  int x = n;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  seg[lane] = x - n;
  const int total = __shfl(x, 63, 64);
  if (lane == 0) seg[64] = total;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  return total;
}

// Parent of each lane's pair in a round of 64 consecutive pairs [c0, c0 + 64)
// of a wave's flattened (parent, candidate) list, where lane k's parent owns
// pairs [start, start + n) (wave_segments' prefix): every non-empty parent
// starting in the round marks its first position (distinct positions), and a
// lane's parent is the last mark at or below it, else `carry`, the parent of
// the previous round's last pair (0 before the first round).  No per-lane walk
// over the prefix.  Called by the whole wave; updates carry.
__device__ __forceinline__ int round_parent(int start, int n, int c0, int *mark, int &carry) {
  const int lane = lane_id();
  mark[lane] = -1;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (n > 0 && start >= c0 && start < c0 + 64) mark[start - c0] = lane;
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int mk = mark[lane];
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const unsigned long long sm = __ballot(mk >= 0) & upto;
  const int from = sm ? 63 - (int)__builtin_clzll(sm) : 0;
  const int got = __shfl(mk, from, 64);
  const int e = sm ? got : carry;
  carry = __builtin_amdgcn_readfirstlane(__shfl(e, 63, 64));
  return e;
}

// Segments of the MDs whose partners the count pass cached: one thread per
// (MD, cache slot), in candidate order, with the angles ls_pass reports.
// kLsCopyLanes threads per MD take slots k, k + kLsCopyLanes, ... (most MDs
// have few segments).
constexpr int kLsCopyLanes = 8;
__global__ void k_ls_copy(const Ws *__restrict__ wb, int keep) {
  const Ws &w = wb[blockIdx.y];
  const long n = (long)uload(w.ctr + C_NMD) * kLsCopyLanes;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int a = (int)(i / kLsCopyLanes), k0 = (int)(i % kLsCopyLanes);
    const int cnt = gp(w.ls_cnt)[a];
    if (cnt > keep) {
      if (k0 == 0) gp(w.ls_ovf)[gp(w.ls_ovf_off)[a]] = a;  // searched again by k_ls_fill
      continue;
    }
    for (int k = k0; k < cnt; k += kLsCopyLanes) {
      const int pos = gp(w.ls_off)[a] + k;
      if (pos >= w.cap_ls) break;
      const int e = gp(w.ls_cache)[(long)a * kLsCache + k];
      const int b = e & 0x3fffffff;
      const float4 B = gload(w.md_pos, b);
      gstore(w.ls_md, pos, make_int2(a, b));
      gstore(w.ls_beta, pos, ls_beta(gload(w.md_pos, a), B));
      gstore(w.ls_opos, pos, B);
      gp(w.ls_oinf)[pos] = (int)((unsigned)e >> 30);
    }
  }
}

// ------------------------------------------------------------- a3: T3
// Parents: segments (a, b); candidates: the segments whose inner MD is b.
// A superset of t3_pass's curvature cut and azimuth-z test (the cuts most
// pairs fail), in the fast operations of the segment pre-tests.  Differences
// from the exact quantities: the curvature and its error within 1e-6
// relative (margin 1e-5); the azimuth-z residual is a difference of two
// products, so its error is bounded by 1e-6 of their magnitudes (margin
// 1e-5 of them) and the tolerance's by 1e-6 relative (margin 1e-5).
__device__ __forceinline__ bool t3_may_pass(const float4 &A, const float4 &B, const float4 &C, ModInfo mA,
                                            ModInfo mB, ModInfo mC, float d0) {
  const float ux = B.x - A.x, uy = B.y - A.y, wx = C.x - A.x, wy = C.y - A.y, tx = C.x - B.x, ty = C.y - B.y;
  const float k = ux * wy - uy * wx;
  const float Lw2 = wx * wx + wy * wy;
  const float kap = (2.0f * k) * (frsq(ux * ux + uy * uy) * frsq(Lw2) * frsq(tx * tx + ty * ty));
  const float dk = (4.0f * ((mA.sig_t() + 2.0f * mB.sig_t()) + mC.sig_t())) * frcp(Lw2);
  if (!(fabsf(kap) <= (kKmaxCut + dk) * 1.00001f)) return false;
  const float su = (A.x * B.y - A.y * B.x) * frcp(A.w * B.w);
  const float sv = (B.x * C.y - B.y * C.x) * frcp(B.w * C.w);
  const float dzpq = B.z - A.z, dzqr = C.z - B.z;
  const float t1 = su * dzqr, t2 = sv * dzpq;
  const float iP = frcp(A.w), iQ = frcp(B.w), iR = frcp(C.w);
  const float ePQ = (mA.hphi() * iP + mB.hphi() * iQ) + d0 * fabsf(iP - iQ);
  const float eQR = (mB.hphi() * iQ + mC.hphi() * iR) + d0 * fabsf(iQ - iR);
  const float au = fabsf(su), av = fabsf(sv), adpq = fabsf(dzpq), adqr = fabsf(dzqr);
  const float nl = (au * au + av * av) * kThird;
  const float tol = ((adqr * ePQ + adpq * eQR) + (au * (mB.ez() + mC.ez()) + av * (mA.ez() + mB.ez()))) +
                    nl * (au * adqr + av * adpq);
  return fabsf(t1 - t2) <= (tol * kMargin + kEps) * 1.00001f + 1e-5f * (fabsf(t1) + fabsf(t2));
}

// First lane of the run of equal values v (lanes 0..n-1 of the wave, runs of
// equal values contiguous) that holds this lane's value.
__device__ __forceinline__ int run_first_lane(int v, int n) {
  const int lane = lane_id();
  const int prev = __shfl_up(v, 1, 64);
  const unsigned long long starts = __ballot(lane < n && (lane == 0 || v != prev));
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  return 63 - __builtin_clzll(starts & upto);
}

// Seven waves per SIMD (at most 72 VGPRs, no spills).
template <bool FILL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) void k_t3(const Ws *__restrict__ wb, DevGeom g) {
  const Ws &w = wb[blockIdx.y];
  __shared__ float4 s_a[kWaves][64], s_b[kWaves][64];
  __shared__ int s_mi[kWaves][64], s_lo[kWaves][64], s_cnt[kWaves][64], s_seg[kWaves][65], s_cached[kWaves][64];
  __shared__ int s_qe[kWaves][128], s_qc[kWaves][128];  // pairs past the pre-test, in pair order
  __shared__ int s_mark[kWaves][64];
  const int n_ls = uload(w.ctr + C_NLS);
  const int wv = wave_id(), lane = lane_id();
  const int wpb = blockDim.x >> 6;
  for (long p0 = ((long)blockIdx.x * wpb + wv) * 64; p0 < n_ls; p0 += (long)gridDim.x * wpb * 64) {
    const int l1 = (int)p0 + lane;
    int n = 0, cached = 0;
    // the fill reads a parent's data only if the count pass found a triplet on it
    if (l1 < n_ls && (!FILL || gp(w.t3_cnt)[l1] > 0)) {
      const int2 ab = gload(w.ls_md, l1);
      s_a[wv][lane] = gload(w.md_pos, ab.x);
      s_b[wv][lane] = gload(w.ls_opos, l1);
      s_mi[wv][lane] = gp(g.info)[gp(w.md_mod)[ab.x]] | (gp(w.ls_oinf)[l1] << 8);
      const int lo = gp(w.ls_off)[ab.y], hi = min(gp(w.ls_off)[ab.y + 1], n_ls);
      s_lo[wv][lane] = lo;
      n = hi > lo ? hi - lo : 0;
      if (FILL) {
        const int cnt = gp(w.t3_cnt)[l1];
        if (cnt <= g.tiles.t3_cache) {  // the count pass kept them all: only those are tested again
          n = cnt;
          cached = 1;
        }
      }
    }
    s_cnt[wv][lane] = 0;
    s_cached[wv][lane] = cached;
    const int total = wave_segments(n, s_seg[wv]);
    // the exact selection on the first nb (<= 64) queued pairs: ranks among each parent's
    // passing pairs from the parent's running count and a ballot over the batch
    auto select = [&](int nb) {
      bool pass = false;
      int e = 0, cand = 0, cmd = 0;
      float4 attr = make_float4(0.f, 0.f, 0.f, 0.f);
      if (lane < nb) {
        e = s_qe[wv][lane];
        cand = s_qc[wv][lane];
        if (FILL) cmd = gload(w.ls_md, cand).y;
        const int mi = s_mi[wv][e];
        pass = t3_pass(s_a[wv][e], s_b[wv][e], gload(w.ls_opos, cand), ModInfo{mi & 0xff}, ModInfo{mi >> 8},
                       ModInfo{gp(w.ls_oinf)[cand]}, &attr, g.d0max);
      }
      const int first = run_first_lane(e, nb);
      const unsigned long long m = __ballot(pass);
      if (pass) {
        const int r = pair_rank(m, first, s_cnt[wv][e]);
        if (!FILL) {
          if (r < g.tiles.t3_cache) gp(w.t3_cache)[(long)((int)p0 + e) * kT3Cache + r] = cand;
        } else {
          const int pos = gp(w.t3_off)[(int)p0 + e] + r;
          if (pos < w.cap_t3) {
            const int2 ab = gload(w.ls_md, (int)p0 + e);
            gstore(w.t3_md, pos, make_int4(ab.x, ab.y, cmd, (int)p0 + e));
            gstore(w.t3_attr, pos, attr);
            gstore(w.t3_first, pos, make_float2(s_a[wv][e].x, s_a[wv][e].y));
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (pass) atomicAdd(&s_cnt[wv][e], 1);  // LDS
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    };
    int nq = 0;
    const int start = s_seg[wv][lane];
    int carry = 0;
    for (int c0 = 0; c0 < total; c0 += 64) {
      const int c = c0 + lane;
      const int e = round_parent(start, n, c0, s_mark[wv], carry);  // parent of this lane's pair
      bool keep = false;
      int cand = 0;
      if (c < total) {
        const int idx = c - s_seg[wv][e];
        cand = s_cached[wv][e] ? gp(w.t3_cache)[(long)((int)p0 + e) * kT3Cache + idx] : s_lo[wv][e] + idx;
        const int mi = s_mi[wv][e];
        keep = t3_may_pass(s_a[wv][e], s_b[wv][e], gload(w.ls_opos, cand), ModInfo{mi & 0xff}, ModInfo{mi >> 8},
                           ModInfo{gp(w.ls_oinf)[cand]}, g.d0max);
      }
      const unsigned long long m = __ballot(keep);
      if (keep) {
        const int q = nq + lanes_below(m);
        s_qe[wv][q] = e;
        s_qc[wv][q] = cand;
      }
      nq += __popcll(m);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (nq >= 64) {
        select(64);
        const int rest = nq - 64;  // < 64: move the queue's tail to its front
        int ve = 0, vc = 0;
        if (lane < rest) {
          ve = s_qe[wv][64 + lane];
          vc = s_qc[wv][64 + lane];
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lane < rest) {
          s_qe[wv][lane] = ve;
          s_qc[wv][lane] = vc;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        nq = rest;
      }
    }
    if (nq > 0) select(nq);
    if (!FILL && l1 < n_ls) gp(w.t3_cnt)[l1] = s_cnt[wv][lane];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// ------------------------------------------------------------- a4: T5
// Parents: triplets (a, b, c); candidates: the triplets whose first MD is c.
// A superset of the azimuth-z test of three anchors (phiz_pass), in the fast
// operations, with the margins of t3_may_pass's azimuth-z part.
__device__ __forceinline__ bool phiz_may_pass(const float4 &P, const float4 &Q, const float4 &R, ModInfo mp,
                                              ModInfo mq, ModInfo mr, float d0) {
  const float su = (P.x * Q.y - P.y * Q.x) * frcp(P.w * Q.w);
  const float sv = (Q.x * R.y - Q.y * R.x) * frcp(Q.w * R.w);
  const float dzpq = Q.z - P.z, dzqr = R.z - Q.z;
  const float t1 = su * dzqr, t2 = sv * dzpq;
  const float iP = frcp(P.w), iQ = frcp(Q.w), iR = frcp(R.w);
  const float ePQ = (mp.hphi() * iP + mq.hphi() * iQ) + d0 * fabsf(iP - iQ);
  const float eQR = (mq.hphi() * iQ + mr.hphi() * iR) + d0 * fabsf(iQ - iR);
  const float au = fabsf(su), av = fabsf(sv), adpq = fabsf(dzpq), adqr = fabsf(dzqr);
  const float nl = (au * au + av * av) * kThird;
  const float tol = ((adqr * ePQ + adpq * eQR) + (au * (mq.ez() + mr.ez()) + av * (mp.ez() + mq.ez()))) +
                    nl * (au * adqr + av * adpq);
  return fabsf(t1 - t2) <= (tol * kMargin + kEps) * 1.00001f + 1e-5f * (fabsf(t1) + fabsf(t2));
}

template <bool FILL>
__global__ __launch_bounds__(kBlock) void k_t5(const Ws *__restrict__ wb, DevGeom g) {
  const Ws &w = wb[blockIdx.y];
  __shared__ float4 s_p[kWaves][3][64], s_tin[kWaves][64];
  __shared__ int s_mi[kWaves][64], s_lo[kWaves][64], s_cnt[kWaves][64], s_seg[kWaves][65], s_cached[kWaves][64];
  __shared__ int s_qe[kWaves][128], s_qc[kWaves][128];  // pairs past the pre-test, in pair order
  const int n_t3 = uload(w.ctr + C_NT3);
  const int n_ls = uload(w.ctr + C_NLS);
  const int wv = wave_id(), lane = lane_id();
  const int wpb = blockDim.x >> 6;
  for (long p0 = ((long)blockIdx.x * wpb + wv) * 64; p0 < n_t3; p0 += (long)gridDim.x * wpb * 64) {
    const int t1 = (int)p0 + lane;
    int n = 0, cached = 0;
    // the fill reads a parent's data only if the count pass found a quintuplet on it
    if (t1 < n_t3 && (!FILL || gp(w.t5_cnt)[t1] > 0)) {
      const int4 abc = gload(w.t3_md, t1);
      s_p[wv][0][lane] = gload(w.md_pos, abc.x);
      s_p[wv][1][lane] = gload(w.md_pos, abc.y);
      s_p[wv][2][lane] = gload(w.md_pos, abc.z);
      s_mi[wv][lane] = gp(g.info)[gp(w.md_mod)[abc.x]] | (g.info[gp(w.md_mod)[abc.y]] << 8) | (g.info[gp(w.md_mod)[abc.z]] << 16);
      s_tin[wv][lane] = gload(w.t3_attr, t1);
      // triplets with first MD c: those built from segments with inner MD c
      const int lsb = min(w.ls_off[abc.z], n_ls), lse = min(w.ls_off[abc.z + 1], n_ls);
      const int lo = gp(w.t3_off)[lsb], hi = min(w.t3_off[lse], n_t3);
      s_lo[wv][lane] = lo;
      n = hi > lo ? hi - lo : 0;
      if (FILL) {
        const int cnt = gp(w.t5_cnt)[t1];
        if (cnt <= g.tiles.t5_cache) {  // the count pass kept them all: only those are tested again
          n = cnt;
          cached = 1;
        }
      }
    }
    s_cnt[wv][lane] = 0;
    s_cached[wv][lane] = cached;
    const int total = wave_segments(n, s_seg[wv]);
    // the exact selection on the first nb (<= 64) queued pairs (as in k_t3)
    auto select = [&](int nb) {
      bool pass = false;
      int e = 0, t2 = 0;
      int4 cde = make_int4(0, 0, 0, 0);
      float at[8];
      if (lane < nb) {
        e = s_qe[wv][lane];
        t2 = s_qc[wv][lane];
        cde = gload(w.t3_md, t2);
        float4 P[5];
        ModInfo M[5];
        const int mi = s_mi[wv][e];
        P[0] = s_p[wv][0][e]; P[1] = s_p[wv][1][e]; P[2] = s_p[wv][2][e];
        M[0].bits = mi & 0xff; M[1].bits = (mi >> 8) & 0xff; M[2].bits = mi >> 16;
        P[3] = gload(w.md_pos, cde.y);
        P[4] = gload(w.md_pos, cde.z);
        M[3].bits = gp(g.info)[gp(w.md_mod)[cde.y]];
        M[4].bits = gp(g.info)[gp(w.md_mod)[cde.z]];
        pass = t5_pass(P, M, s_tin[wv][e], gload(w.t3_attr, t2), at, g.d0max, g.t5cut);
      }
      const int first = run_first_lane(e, nb);
      const unsigned long long m = __ballot(pass);
      if (pass) {
        const int r = pair_rank(m, first, s_cnt[wv][e]);
        if (!FILL) {
          if (r < g.tiles.t5_cache) gp(w.t5_cache)[(long)((int)p0 + e) * kT5Cache + r] = t2;
        } else {
          const int t1e = (int)p0 + e;
          const int pos = gp(w.t5_off)[t1e] + r;
          if (pos < w.cap_t5) {
            const int4 abc = gload(w.t3_md, t1e);
            gstore(w.t5_t3, pos, make_int2(t1e, t2));
            int *md = w.t5_md + 5 * (long)pos;
            md[0] = abc.x; md[1] = abc.y; md[2] = abc.z; md[3] = cde.y; md[4] = cde.z;
            float *dst = w.t5_attr + 8 * (long)pos;
#pragma unroll
            for (int k = 0; k < 8; ++k) dst[k] = at[k];
            gp(w.t5_keep)[pos] = 1;  // until a better duplicate is found
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (pass) atomicAdd(&s_cnt[wv][e], 1);  // LDS
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    };
    int nq = 0;
    int e = 0;  // parent of this lane's pair (pairs advance monotonically; the walk keeps registers
                // low enough for five waves per SIMD)
    for (int c0 = 0; c0 < total; c0 += 64) {
      const int c = c0 + lane;
      bool keep = false;
      int t2 = 0;
      if (c < total) {
        while (s_seg[wv][e + 1] <= c) ++e;
        const int idx = c - s_seg[wv][e];
        t2 = s_cached[wv][e] ? gp(w.t5_cache)[(long)((int)p0 + e) * kT5Cache + idx] : s_lo[wv][e] + idx;
        // the radius compatibility cut exactly (no division), then the fast azimuth-z test
        const float4 tin = s_tin[wv][e], tout = gload(w.t3_attr, t2);
        if (fabsf(tin.x - tout.x) <= tin.y + tout.y) {
          const int4 cde = gload(w.t3_md, t2);
          const int mi = s_mi[wv][e];
          keep = phiz_may_pass(s_p[wv][0][e], s_p[wv][2][e], gload(w.md_pos, cde.z), ModInfo{mi & 0xff},
                               ModInfo{mi >> 16}, ModInfo{gp(g.info)[gp(w.md_mod)[cde.z]]}, g.d0max);
        }
      }
      const unsigned long long m = __ballot(keep);
      if (keep) {
        const int q = nq + lanes_below(m);
        s_qe[wv][q] = e;
        s_qc[wv][q] = t2;
      }
      nq += __popcll(m);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (nq >= 64) {
        select(64);
        const int rest = nq - 64;
        int ve = 0, vc = 0;
        if (lane < rest) {
          ve = s_qe[wv][64 + lane];
          vc = s_qc[wv][64 + lane];
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lane < rest) {
          s_qe[wv][lane] = ve;
          s_qc[wv][lane] = vc;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        nq = rest;
      }
    }
    if (nq > 0) select(nq);
    if (!FILL && t1 < n_t3) gp(w.t5_cnt)[t1] = s_cnt[wv][lane];
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// ------------------------------------------------------------- a5: T5 dedup
__global__ void k_t5_inc_count(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = uload(w.ctr + C_NT5);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    for (int k = 0; k < 5; ++k) atomicAdd(&w.inc_cnt[gp(w.t5_md)[5 * (long)t + k]], 1);
}
__global__ void k_t5_inc_scatter(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = uload(w.ctr + C_NT5);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int score = __float_as_int(w.t5_attr[8 * (long)t + 1]);
    for (int k = 0; k < 5; ++k) {
      const int md = gp(w.t5_md)[5 * (long)t + k];
      w.inc_list[gp(w.inc_off)[md] + atomicAdd(&w.inc_cur[md], 1)] = make_int2(t, score);
    }
  }
}

__device__ __forceinline__ void t5_hits(const Ws &w, int t, int *h) {
  const int *md = w.t5_md + 5 * (long)t;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const int2 hh = w.md_hits[md[k]];
    h[2 * k] = hh.x;
    h[2 * k + 1] = hh.y;
  }
}
// (score, tuple) of u strictly smaller than (score, tuple) of t
template <int N>
__device__ __forceinline__ bool better(float su, const int *hu, float st, const int *ht) {
  if (su < st) return true;
  if (st < su) return false;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (hu[k] < ht[k]) return true;
    if (ht[k] < hu[k]) return false;
  }
  return false;
}

// A T5 is dropped when another T5 sharing at least two MDs has a smaller (chi2_xy, hit tuple).
// Items (T5 t, k < 4); an item's candidates are the T5s u listed at t's k-th
// MD, and u is judged there only if it shares at least two MDs with t and its
// first MD in common with t's first four is that k-th one (so each pair is
// judged once; a duplicate shares two of the five MDs, hence one of the first
// four).  Flattened as in the T3/T5 searches: a wave takes ipw items (64, or
// 16 when one event alone leaves too few waves to hide the gathers' latency),
// stages their MDs in LDS and strides all (item, candidate) pairs with its
// lanes.
// t5_keep starts at 1 (written by the fill); a strictly better duplicate
// clears it (every writer writes 0).
// Its LDS is dynamic, kT5DedupLds bytes per wave of the block, so that a tuned
// launch of one-wave blocks does not hold four waves' worth.
struct T5DedupLds {
  int mt[5][64], lo[64], seg[65], mark[64];
  float st[64];
};
constexpr size_t kT5DedupLds = sizeof(T5DedupLds);

__global__ __launch_bounds__(kBlock) void k_t5_dedup(const Ws *__restrict__ wb, int ipw) {
  extern __shared__ T5DedupLds s_dd[];
  const Ws &w = wb[blockIdx.y];
  const int n = uload(w.ctr + C_NT5);
  const int wv = wave_id(), lane = lane_id();
  const int wpb = blockDim.x >> 6;
  auto &S = s_dd[wv];
  for (long p0 = ((long)blockIdx.x * wpb + wv) * ipw; p0 < 4L * n; p0 += (long)gridDim.x * wpb * ipw) {
    const long item = p0 + lane;
    int cnt = 0;
    if (lane < ipw && item < 4L * n) {
      const int t = (int)(item >> 2), k = (int)(item & 3);
      int mt[5];
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        mt[j] = gp(w.t5_md)[5 * (long)t + j];
        S.mt[j][lane] = mt[j];
      }
      if (k == 0) gstore(w.t5_first, t, make_float2(w.md_pos[mt[0]].x, w.md_pos[mt[0]].y));
      const int lo = gp(w.inc_off)[mt[k]];
      S.lo[lane] = lo;
      cnt = gp(w.inc_off)[mt[k] + 1] - lo;
      S.st[lane] = gp(w.t5_attr)[8 * (long)t + 1];
    }
    const int total = wave_segments(cnt, S.seg);
    const int start = S.seg[lane];
    int carry = 0;
    for (int c0 = 0; c0 < total; c0 += 64) {
      const int c = c0 + lane;
      const int e = round_parent(start, cnt, c0, S.mark, carry);  // item of this lane's pair
      if (c >= total) continue;
      const int t = (int)((p0 + e) >> 2), k = (int)((p0 + e) & 3);
      const int2 ue = w.inc_list[S.lo[e] + (c - S.seg[e])];
      const int u = ue.x;
      if (u == t) continue;
      // only a u that is not worse can drop t: the score first (kept in the list entry),
      // then sharing, then on a tie of scores the hit tuples (the decision of better<10>)
      const float su = __int_as_float(ue.y), st = S.st[e];
      if (st < su) continue;
      int mu[5];
#pragma unroll
      for (int j = 0; j < 5; ++j) mu[j] = gp(w.t5_md)[5 * (long)u + j];
      int shared = 0, first = 5;
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const int v = S.mt[j][e];
        const bool in = v == mu[0] || v == mu[1] || v == mu[2] || v == mu[3] || v == mu[4];
        shared += in ? 1 : 0;
        first = (in && first == 5) ? j : first;
      }
      if (shared < 2 || first != k) continue;
      bool drop = su < st;
      if (!drop) {
        int ht[10], hu[10];
        t5_hits(w, t, ht);
        t5_hits(w, u, hu);
        drop = better<10>(su, hu, st, ht);
      }
      if (drop) gp(w.t5_keep)[t] = 0;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// ------------------------------------------------------------- a6: pLS
__device__ __forceinline__ Seed load_seed(const Ws &w, int s) {
  const float *p = w.pls + 8 * (long)s;
  Seed sd;
  sd.pt = p[0]; sd.cx = p[1]; sd.cy = p[2]; sd.lam = p[3]; sd.ks = p[4]; sd.x0 = p[5]; sd.y0 = p[6]; sd.z0 = p[7];
  return sd;
}

__global__ void k_pls(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < w.n_seeds; s += gridDim.x * blockDim.x) {
    const float px = gp(w.px)[s], py = gp(w.py)[s], pz = gp(w.pz)[s];
    const float pt = sqrtf(px * px + py * py);
    float *o = w.pls + 8 * (long)s;
    o[0] = pt;
    o[1] = px / pt;
    o[2] = py / pt;
    o[3] = pz / pt;
    o[4] = (-(float)gp(w.q)[s] * kCurv) / pt;
    int h0 = gp(w.hits4)[4 * (long)s];
    h0 = (h0 >= 0 && h0 < w.n_hits) ? h0 : 0;
    o[5] = gp(w.x)[h0];
    o[6] = gp(w.y)[h0];
    o[7] = gp(w.z)[h0];
    for (int k = 0; k < 4; ++k) {
      const int h = gp(w.hits4)[4 * (long)s + k];
      if (h >= 0 && h < w.n_hits) atomicAdd(&w.ph_cnt[h], 1);
    }
  }
}
__global__ void k_ph_scatter(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < w.n_seeds; s += gridDim.x * blockDim.x)
    for (int k = 0; k < 4; ++k) {
      const int h = gp(w.hits4)[4 * (long)s + k];
      if (h >= 0 && h < w.n_hits) gp(w.ph_list)[gp(w.ph_off)[h] + atomicAdd(&w.ph_cur[h], 1)] = s;
    }
}
// pLS duplicate removal: seeds sharing at least 3 pixel hits; the lower seed index wins.
__global__ void k_pls_dedup(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < w.n_seeds; s += gridDim.x * blockDim.x) {
    int hs[4];
    for (int k = 0; k < 4; ++k) hs[k] = gp(w.hits4)[4 * (long)s + k];
    bool keep = true;
    for (int k = 0; k < 4 && keep; ++k) {
      const int h = hs[k];
      if (h < 0 || h >= w.n_hits) continue;
      for (int q = gp(w.ph_off)[h]; q < gp(w.ph_off)[h + 1] && keep; ++q) {
        const int t = gp(w.ph_list)[q];
        if (t >= s) continue;
        int sh = 0;
        for (int i = 0; i < 4; ++i) {
          const int hi = hs[i];
          bool f = false;
          for (int j = 0; j < 4; ++j) f |= (w.hits4[4 * (long)t + j] == hi);
          sh += f ? 1 : 0;
        }
        if (sh >= 3) keep = false;
      }
    }
    gp(w.pls_keep)[s] = keep ? 1 : 0;
  }
}

// ------------------------------------------------------------- a7: pT3 / pT5
template <int K>
__device__ __forceinline__ void load_object(const Ws &w, const DevGeom &g, int t, float4 *P, ModInfo *M, float *kT,
                                            float *dkT) {
  if constexpr (K == 3) {
    const int4 abc = gload(w.t3_md, t);
    const int md[3] = {abc.x, abc.y, abc.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) { P[k] = w.md_pos[md[k]]; M[k].bits = gp(g.info)[gp(w.md_mod)[md[k]]]; }
    const float4 a3 = gload(w.t3_attr, t);
    *kT = a3.x; *dkT = a3.y;
  } else {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int md = gp(w.t5_md)[5 * (long)t + k];
      P[k] = gload(w.md_pos, md);
      M[k].bits = gp(g.info)[gp(w.md_mod)[md]];
    }
    const float4 a3 = w.t3_attr[gload(w.t5_t3, t).y];
    *kT = a3.x; *dkT = a3.y;
  }
}

// ---- binned search: objects grouped by first anchor (radius ring, azimuth bin, z bin)
constexpr int kRings = 10;
constexpr float kRing0 = 20.0f, kRingW = 10.0f;      // rings [20, 30), ..., [110, 120) cm, ends clamped
constexpr int kPhiBins = 256;
constexpr int kObjBins = kRings * kPhiBins;          // (ring, azimuth) pairs: the bits of a seed's mask
constexpr int kZBins = 55;
constexpr float kZHalf = 275.0f, kZW = 10.0f;        // z bins [-275, -265), ..., ends clamped
static_assert(kObjBins * kZBins == kSeedBins, "seed-search bin count");
constexpr int kMaskWords = kObjBins / 32;
constexpr float kSampleStep = 2.0f;                  // trajectory sampling step [cm]
constexpr int kMaxSamples = 112;                     // 224 cm of arc

__device__ __forceinline__ int ring_of(float r) {
  const int k = (int)floorf((r - kRing0) / kRingW);
  return k < 0 ? 0 : (k >= kRings ? kRings - 1 : k);
}
__device__ __forceinline__ int phibin_of(float ph) {
  const int b = (int)floorf((ph + (float)M_PI) * (float)(kPhiBins / (2.0 * M_PI)));
  return b < 0 ? 0 : (b >= kPhiBins ? kPhiBins - 1 : b);
}
__device__ __forceinline__ int zbin_of(float z) {
  const int b = (int)floorf((z + kZHalf) / kZW);
  return b < 0 ? 0 : (b >= kZBins ? kZBins - 1 : b);
}
template <int K>
__device__ __forceinline__ int obj_bin(const Ws &w, int t) {
  const float4 a = w.md_pos[K == 3 ? gload(w.t3_md, t).x : gp(w.t5_md)[5 * (long)t]];
  const float ph = atan2f(a.y, a.x);
  const int rp = ph == ph ? ring_of(sqrtf(a.x * a.x + a.y * a.y)) * kPhiBins + phibin_of(ph) : 0;
  return rp * kZBins + zbin_of(a.z);
}

template <int K>
__global__ void k_obj_bin_count(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = K == 3 ? w.ctr[C_NT3] : w.ctr[C_NT5];
  int *cnt = K == 3 ? w.b3_cnt : w.b5_cnt;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    if (K == 3 || gp(w.t5_keep)[t]) atomicAdd(&cnt[obj_bin<K>(w, t)], 1);
}
template <int K>
__global__ void k_obj_bin_scatter(const Ws *__restrict__ wb, DevGeom g) {
  const Ws &w = wb[blockIdx.y];
  const int n = K == 3 ? w.ctr[C_NT3] : w.ctr[C_NT5];
  const int *off = K == 3 ? w.b3_off : w.b5_off;
  int *cur = K == 3 ? w.b3_cur : w.b5_cur;
  int *lst = K == 3 ? w.b3_list : w.b5_list;
  float4 *pos = K == 3 ? w.b3_pos : w.b5_pos;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    if (K == 3 || gp(w.t5_keep)[t]) {
      const int b = obj_bin<K>(w, t);
      const int j = off[b] + atomicAdd(&cur[b], 1);
      lst[j] = t;
      const int md = K == 3 ? gload(w.t3_md, t).x : gp(w.t5_md)[5 * (long)t];
      const float4 a = gload(w.md_pos, md);
      pos[j] = make_float4(a.x, a.y, a.z, __int_as_float(g.info[gp(w.md_mod)[md]]));
    }
}

// Processing order of the seed search: seeds grouped by direction (azimuth of
// the seed's direction in kPhiBins sectors x 8 bins of lambda), one block of
// 1024 threads per event.  Seeds of one group scan nearly the same bins, so
// waves that run together (consecutive blocks) reuse each other's object
// lists in cache.  Results do not depend on the order (each seed writes only
// its own entries), so ranks within a group come from LDS atomics.
constexpr int kSeedKeys = kPhiBins * 8;
__device__ __forceinline__ int seed_key(const Ws &w, int s) {
  const float *p = w.pls + 8 * (long)s;
  const float ph = atan2f(p[2], p[1]);
  const int lb = (int)floorf((p[3] + 6.0f) * (1.0f / 1.5f));
  return (ph == ph ? phibin_of(ph) : 0) * 8 + (lb < 0 ? 0 : (lb > 7 ? 7 : lb));
}
constexpr int kSeedKeyLds = 10240;  // seeds whose key the ordering keeps in LDS (the rest recompute it)
__global__ __launch_bounds__(1024) void k_seed_order(const Ws *__restrict__ wb) {
  __shared__ int s_cnt[kSeedKeys];
  __shared__ unsigned short s_key[kSeedKeyLds];
  __shared__ int s_wave[16];
  static_assert(kSeedKeys <= 65536, "a key fits 16 bits");
  const Ws &w = wb[blockIdx.y];
  const int S = w.n_seeds, t = threadIdx.x, lane = lane_id(), wv = t >> 6;
  for (int k = t; k < kSeedKeys; k += 1024) s_cnt[k] = 0;
  __syncthreads();
  for (int s = t; s < S; s += 1024) {
    const int key = seed_key(w, s);
    if (s < kSeedKeyLds) s_key[s] = (unsigned short)key;
    atomicAdd(&s_cnt[key], 1);  // LDS
  }
  __syncthreads();
  // exclusive scan of the key counts: two keys per thread, then over the block
  static_assert(kSeedKeys == 2 * 1024, "two keys per thread");
  const int c0 = s_cnt[2 * t], c1 = s_cnt[2 * t + 1];
  int x = c0 + c1;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_wave[wv] = x;
  __syncthreads();
  int before = 0;
  for (int q = 0; q < wv; ++q) before += s_wave[q];
  const int ex = before + x - (c0 + c1);
  s_cnt[2 * t] = ex;
  s_cnt[2 * t + 1] = ex + c0;
  __syncthreads();
  for (int s = t; s < S; s += 1024) {
    const int key = s < kSeedKeyLds ? (int)s_key[s] : seed_key(w, s);
    gp(w.seed_order)[atomicAdd(&s_cnt[key], 1)] = s;  // LDS rank
  }
}

// Marks, in the wave's bin mask, every (ring, azimuth) bin that can hold the
// first anchor of an object inside the seed's window: the anchor lies within
// 1.01 cm of the seed circle on its forward half-turn (algebraic distance
// <= 1 cm with |kappa| <= 0.02/cm), hence within d = 1.01 + step/2 + 0.05 cm
// of a trajectory sample taken every `kSampleStep` of arc.
static_assert(kPhiBins % 32 == 0, "a ring's row of the bin mask is whole words");

// Sets bits id0 .. id0 + n - 1 of the mask, one atomic per word.
__device__ __forceinline__ void mark_run(unsigned *mask, int id0, int n) {
  const int end = id0 + n;
  for (int id = id0; id < end;) {
    const int bit = id & 31;
    const int take = min(32 - bit, end - id);
    const unsigned m = take == 32 ? 0xffffffffu : ((1u << take) - 1u) << bit;
    atomicOr(&mask[id >> 5], m);
    id += take;
  }
}

__device__ void mark_seed_bins(const Seed &sd, unsigned *mask, int *s_lo, int *s_hi) {
  const int lane = lane_id();
  const float d = 1.01f * kBoxXY + 0.5f * kSampleStep + 0.05f;
  const float bw = (float)(2.0 * M_PI / kPhiBins);
  const float k = sd.ks;
  const float ak = fabsf(k) > 1e-9f ? fabsf(k) : 1e-9f;
  const float s_max = (float)M_PI / ak;
  const float px = -sd.cy, py = sd.cx;  // perpendicular of the direction
  for (int i = lane; i < kMaxSamples; i += 64) {
    const float sarc = i * kSampleStep;
    if (sarc > s_max + kSampleStep) continue;
    const float a = k * sarc;
    const float s1 = fabsf(k) > 1e-9f ? sinf(a) / k : sarc;
    const float sh = sinf(0.5f * a);
    const float s2 = fabsf(k) > 1e-9f ? 2.0f * sh * sh / k : 0.0f;
    const float x = sd.x0 + sd.cx * s1 + px * s2;
    const float y = sd.y0 + sd.cy * s1 + py * s2;
    const float r = sqrtf(x * x + y * y);
    if (r + d < kRing0 - 5.0f || r - d > kRing0 + kRings * kRingW + 5.0f) continue;
    const int r0 = ring_of(r - d), r1 = ring_of(r + d);
    const float rin = r - d;
    int b0, b1;
    if (rin <= 1e-3f || d / rin >= 1.0f) {
      b0 = 0;
      b1 = kPhiBins - 1;
    } else {
      // an anchor within d of the sample, at radius >= rin, is within asin(d / rin) of
      // its azimuth; 2e-4 rad (1% of a bin) covers the rounding of these bin edges
      // against phibin_of's
      const float hw = asinf(d / rin);
      const float ph = atan2f(y, x);
      b0 = (int)floorf((ph - hw - 2e-4f + (float)M_PI) / bw);
      b1 = (int)floorf((ph + hw + 2e-4f + (float)M_PI) / bw);
      if (b1 - b0 >= kPhiBins) { b0 = 0; b1 = kPhiBins - 1; }
    }
    // bins b0..b1 (fewer than kPhiBins, may wrap round) as at most two runs of
    // one ring's row; a ring's row is whole mask words, so each word a run
    // touches takes one atomic
    const int lo = ((b0 % kPhiBins) + kPhiBins) % kPhiBins;
    const int len = b1 - b0 + 1;
    const int n1 = min(len, kPhiBins - lo);
    for (int rr = r0; rr <= r1; ++rr) {
      // arc lengths are >= 0, so their float bits order like ints
      atomicMin(&s_lo[rr], __float_as_int(sarc));
      atomicMax(&s_hi[rr], __float_as_int(sarc));
      mark_run(mask, rr * kPhiBins + lo, n1);
      if (len > n1) mark_run(mask, rr * kPhiBins, len - n1);
    }
  }
}

// z bins of ring rr that can hold the first anchor of an object inside the
// seed's window, from the arc-length range [lo, hi] of the samples that marked
// the ring: the anchor's arc length from the seed hit (the chord series of
// pt_pass) is within d + step + 1.5 cm of such a sample's, and its z within
// the first-anchor z window (3 cm + 2 sigma_z, sigma_z at most
// max(2.5, 2.5 |lambda| + 0.01) cm) of z0 + lambda s; margins on top.
__device__ __forceinline__ int2 seed_zbins(const Seed &sd, float lo, float hi) {
  const float ds = 1.01f * kBoxXY + 1.5f * kSampleStep + 1.6f;
  const float al = fabsf(sd.lam);
  const float zw = (kBoxZ0 + 2.0f * fmaxf(2.5f, 2.5f * al + 0.01f)) * 1.01f + 0.1f;
  const float za = sd.z0 + sd.lam * (lo - ds), zb = sd.z0 + sd.lam * (hi + ds);
  return make_int2(zbin_of(fminf(za, zb) - zw), zbin_of(fmaxf(za, zb) + zw));
}

// One wave per seed over the objects of the bins its trajectory can reach.
// COUNT: number of passing objects.  FILL: passing object indices gathered in
// LDS, ranked by object index, written at the seed's offset in object order
// (the order of the full scan); a seed with more passing objects than the
// list holds (tile pass_list <= kPassList) is filled by an ordered scan over
// all objects instead.  The count pass keeps up to pt3_cache / pt5_cache
// passing objects per seed with their attributes, which the fill then ranks
// and copies; more than max_slices marked bins are searched bin by bin.
// (Seven waves per SIMD for the count: at most 72 VGPRs, no spills.)
template <int K, bool FILL, bool BOTH = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) void k_pt_binned(const Ws *__restrict__ wb, DevGeom g) {
  __shared__ unsigned s_mask[kWaves][kMaskWords];
  __shared__ int s_slo[kWaves][kRings], s_shi[kWaves][kRings];
  __shared__ int2 s_zb[kWaves][kRings];
  __shared__ int s_sl_j0[kWaves][kMaxSlices];       // bin id of each slice, then first list entry of each slice with candidates
  __shared__ int s_sl_pre[kWaves][kMaxSlices];      // candidates before each slice with candidates
  __shared__ int s_list[FILL ? kWaves : 1][FILL ? kPassList : 1];
  __shared__ int s_pq[kWaves][128];  // candidates past the first-anchor test, awaiting the full one
  __shared__ int s_mark[kWaves][64];  // a slice's candidates start here (this round)
  const Ws &w = wb[blockIdx.y];
  const int wv = wave_id(), lane = lane_id();
  const int si = blockIdx.x * (int)(blockDim.x >> 6) + wv;
  if (si >= w.n_seeds) return;
  const int s = uload(w.seed_order + si);  // seeds of one direction on neighbouring waves
  const Seed sd = load_seed(w, s);
  constexpr int kCache = K == 3 ? kPt3Cache : kPt5Cache;
  static_assert(kCache <= kPassList, "the fill ranks the cache in its LDS list");
  const int keep = K == 3 ? g.tiles.pt3_cache : g.tiles.pt5_cache;  // <= kCache
  const int pass_list = g.tiles.pass_list;                            // <= kPassList
  const int max_slices = g.tiles.max_slices;                          // <= kMaxSlices
  int *cache = (K == 3 ? w.pt3_cache : w.pt5_cache) + (long)s * kCache;
  float4 *cattr = (K == 3 ? w.pt3_cattr : w.pt5_cattr) + (long)s * kCache;
  if constexpr (FILL) {
    // the count pass cached every passing object of this seed with its attributes:
    // rank them by object index (in LDS) and copy, no search
    const int expect = (K == 3 ? w.pt3_cnt : w.pt5_cnt)[s];
    if (expect <= keep) {
      for (int i = lane; i < expect; i += 64) s_list[wv][i] = cache[i];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      for (int i = lane; i < expect; i += 64) {
        const int t = s_list[wv][i];
        int rank = 0;
        for (int q = 0; q < expect; ++q) rank += s_list[wv][q] < t ? 1 : 0;
        const int pos = (K == 3 ? w.pt3_off : w.pt5_off)[s] + rank;
        if (pos < (K == 3 ? w.cap_pt3 : w.cap_pt5)) {
          (K == 3 ? w.pt3_so : w.pt5_so)[pos] = make_int2(s, t);
          (K == 3 ? w.pt3_attr : w.pt5_attr)[pos] = cattr[i];
        }
      }
      return;
    }
  }
  unsigned *mask = s_mask[wv];
  for (int i = lane; i < kMaskWords; i += 64) mask[i] = 0u;
  if (lane < kRings) {
    s_slo[wv][lane] = 0x7f7fffff;  // largest finite float
    s_shi[wv][lane] = 0;
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  mark_seed_bins(sd, mask, s_slo[wv], s_shi[wv]);
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (lane < kRings)
    s_zb[wv][lane] = seed_zbins(sd, __int_as_float(s_slo[wv][lane]), __int_as_float(s_shi[wv][lane]));
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // the search over one object kind's bins (KO = 3: triplets, 5: quintuplets)
  auto search = [&](auto kind) {
    constexpr int KO = decltype(kind)::value;
    constexpr int kCacheO = KO == 3 ? kPt3Cache : kPt5Cache;
    const int keepO = KO == 3 ? g.tiles.pt3_cache : g.tiles.pt5_cache;
    int *cache = (KO == 3 ? w.pt3_cache : w.pt5_cache) + (long)s * kCacheO;
    float4 *cattr = (KO == 3 ? w.pt3_cattr : w.pt5_cattr) + (long)s * kCacheO;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int *boff = KO == 3 ? w.b3_off : w.b5_off;
    const int *blst = KO == 3 ? w.b3_list : w.b5_list;
    const float2 *first = KO == 3 ? w.t3_first : w.t5_first;
    int n_pass = 0;
    int base = FILL ? (KO == 3 ? w.pt3_off : w.pt5_off)[s] : 0;
    const int expect = FILL ? (KO == 3 ? w.pt3_cnt : w.pt5_cnt)[s] : 0;
    const int cap = KO == 3 ? w.cap_pt3 : w.cap_pt5;
    const bool listed = !FILL || expect <= pass_list;
    const float4 *bpos = KO == 3 ? w.b3_pos : w.b5_pos;
    // the full selection on the first n (<= 64) queued objects; passing ones are counted
    // in ballot order and remembered (count: the cache; fill: the LDS list)
    auto full = [&](int n) {
      bool pass = false;
      int t = 0;
      float4 attr = make_float4(0.f, 0.f, 0.f, 0.f);
      if (lane < n) {
        t = s_pq[wv][lane];
        float4 P[KO];
        ModInfo M[KO];
        float kT, dkT;
        load_object<KO>(w, g, t, P, M, &kT, &dkT);
        pass = pt_pass<KO>(sd, P, M, kT, dkT, &attr);
      }
      const unsigned long long m = __ballot(pass);
      if (pass) {
        const int pre = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
        if (FILL) {
          if (n_pass + pre < kPassList) s_list[wv][n_pass + pre] = t;
        } else if (n_pass + pre < keepO) {
          cache[n_pass + pre] = t;
          cattr[n_pass + pre] = attr;
        }
      }
      n_pass += __popcll(m);
    };
    // one candidate per lane (list entry j): the exact first-anchor part of the selection
    // from the packed anchor; objects passing it are queued, and the full selection runs
    // on full waves of them
    int nq = 0;
    auto test = [&](bool active, int j) {
      bool keep = false;
      int t = 0;
      if (active) {
        t = blst[j];
        const float4 f = bpos[j];
        keep = pt_first_anchor(sd, f, ModInfo{__float_as_int(f.w)});
      }
      const unsigned long long m = __ballot(keep);
      if (keep)
        s_pq[wv][nq + __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u))] = t;
      nq += __popcll(m);
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      if (nq >= 64) {
        full(64);
        const int rest = nq - 64;  // < 64: move the queue's tail to its front
        const int v = lane < rest ? s_pq[wv][64 + lane] : 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (lane < rest) s_pq[wv][lane] = v;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        nq = rest;
      }
    };
    bool flat = false;
    if (listed) {
      // every marked (ring, azimuth) bin becomes a slice of the object list (its reachable
      // z bins, possibly empty); bit ids first, ranked over the wave by a prefix of the
      // mask words' popcounts, then converted in place, 64 at a time, to (first entry,
      // candidates before it)
      int n_bits = 0;
      for (int w0 = 0; w0 < kMaskWords; w0 += 64) {
        const unsigned bits = w0 + lane < kMaskWords ? s_mask[wv][w0 + lane] : 0u;
        const int pc = __popc(bits);
        int x = pc;
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(x, o, 64);
          if (lane >= o) x += y;
        }
        const int tot = __shfl(x, 63, 64);
        if (n_bits + tot <= max_slices) {
          int k = n_bits + x - pc;
          for (unsigned bb = bits; bb; bb &= bb - 1u) s_sl_j0[wv][k++] = (w0 + lane) * 32 + __builtin_ctz(bb);
        }
        n_bits += tot;
      }
      flat = n_bits <= max_slices;
      if (flat) {
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // slices with candidates only, compacted in place (an entry is read before any
        // write of its round, and compacted positions never pass the round's own)
        int run = 0, n_live = 0;
        for (int c0 = 0; c0 < n_bits; c0 += 64) {
          const int k = c0 + lane;
          int j0 = 0, len = 0;
          if (k < n_bits) {
            const int bin = s_sl_j0[wv][k];
            const int2 zb = s_zb[wv][bin / kPhiBins];
            j0 = boff[bin * kZBins + zb.x];
            len = boff[bin * kZBins + zb.y + 1] - j0;
          }
          int x = len;
          for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
          }
          const unsigned long long live = __ballot(len > 0);
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
          __builtin_amdgcn_wave_barrier();
          if (len > 0) {
            const int q = n_live + lanes_below(live);
            s_sl_j0[wv][q] = j0;
            s_sl_pre[wv][q] = run + x - len;
          }
          n_live += __popcll(live);
          run += __builtin_amdgcn_readfirstlane(__shfl(x, 63, 64));
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // the slice of each lane's candidate: the slices starting before the round (jlo)
        // plus those starting at or below the lane in it (distinct starts, marked)
        int jlo = 0;
        for (int c0 = 0; c0 < run; c0 += 64) {
          const int c = c0 + lane;
          s_mark[wv][lane] = 0;
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
          __builtin_amdgcn_wave_barrier();
          if (jlo + lane < n_live) {
            const int p = s_sl_pre[wv][jlo + lane] - c0;  // >= 0
            if (p < 64) s_mark[wv][p] = 1;
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
          __builtin_amdgcn_wave_barrier();
          const unsigned long long starts = __ballot(s_mark[wv][lane] != 0);
          int j = 0;
          if (c < run) {
            const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
            const int e = jlo - 1 + __popcll(starts & upto);
            j = s_sl_j0[wv][e] + (c - s_sl_pre[wv][e]);
          }
          jlo += __popcll(starts);
          test(c < run, j);
        }
      }
    }
    if (listed && !flat) {
      n_pass = 0;
      nq = 0;
      for (int wd = 0; wd < kMaskWords; ++wd) {
        unsigned bits = mask[wd];
        while (bits) {
          const int bit = __builtin_ctz(bits);
          bits &= bits - 1u;
          const int bin = wd * 32 + bit;
          const int2 zb = s_zb[wv][bin / kPhiBins];
          const int j0 = boff[bin * kZBins + zb.x], j1 = boff[bin * kZBins + zb.y + 1];
          for (int j = j0 + lane; j - lane < j1; j += 64) test(j < j1, j);
        }
      }
    }
    if (listed && nq > 0) full(nq);
    if (!FILL) {
      if (lane == 0) (KO == 3 ? w.pt3_cnt : w.pt5_cnt)[s] = n_pass;
      return;
    }
    if (listed) {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // rank by object index (indices are distinct) and write in object order
      for (int i = lane; i < n_pass; i += 64) {
        const int t = s_list[wv][i];
        int rank = 0;
        for (int q = 0; q < n_pass; ++q) rank += s_list[wv][q] < t ? 1 : 0;
        const int pos = base + rank;
        if (pos < cap) {
          float4 P[KO];
          ModInfo M[KO];
          float kT, dkT;
          float4 attr;
          load_object<KO>(w, g, t, P, M, &kT, &dkT);
          pt_pass<KO>(sd, P, M, kT, dkT, &attr);
          (KO == 3 ? w.pt3_so : w.pt5_so)[pos] = make_int2(s, t);
          (KO == 3 ? w.pt3_attr : w.pt5_attr)[pos] = attr;
        }
      }
      return;
    }
    // rare: too many passing objects for the LDS list; ordered scan of all objects
    const int n_obj = KO == 3 ? w.ctr[C_NT3] : w.ctr[C_NT5];
    for (int t0 = 0; t0 < n_obj; t0 += 64) {
      const int t = t0 + lane;
      bool pass = false;
      float4 attr = make_float4(0.f, 0.f, 0.f, 0.f);
      if (t < n_obj && (KO == 3 || gp(w.t5_keep)[t])) {
        const float2 f = first[t];
        if (seed_box(sd, f.x, f.y)) {
          float4 P[KO];
          ModInfo M[KO];
          float kT, dkT;
          load_object<KO>(w, g, t, P, M, &kT, &dkT);
          pass = pt_pass<KO>(sd, P, M, kT, dkT, &attr);
        }
      }
      const unsigned long long m = __ballot(pass);
      const int pre = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
      if (pass && base + pre < cap) {
        (KO == 3 ? w.pt3_so : w.pt5_so)[base + pre] = make_int2(s, t);
        (KO == 3 ? w.pt3_attr : w.pt5_attr)[base + pre] = attr;
      }
      base += __popcll(m);
    }
  };
  if constexpr (BOTH) {  // count pass of both kinds on one trajectory mask
    search(std::integral_constant<int, 3>{});
    search(std::integral_constant<int, 5>{});
  } else {
    search(std::integral_constant<int, K>{});
  }
}

// The key that orders a pT entry for the same-object rule: smaller (score,
// seed) is better, and since scores are >= 0 their bits order them as
// integers; complemented so that the best is the largest, found with an
// atomic maximum per outer object (a value, not a position: order-independent).
template <int K>
__device__ __forceinline__ unsigned long long pt_obj_key(const Ws &w, int i) {
  const float4 *at = K == 3 ? w.pt3_attr : w.pt5_attr;
  const int2 *so = K == 3 ? w.pt3_so : w.pt5_so;
  return ~(((unsigned long long)__float_as_uint(at[i].z) << 32) | (unsigned long long)(unsigned)so[i].x);
}
template <int K>
__global__ void k_pt_obj_best(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = K == 3 ? w.ctr[C_NPT3] : w.ctr[C_NPT5];
  const int2 *so = K == 3 ? w.pt3_so : w.pt5_so;
  unsigned long long *best = K == 3 ? w.o3_best : w.o5_best;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    atomicMax(&best[so[i].y], pt_obj_key<K>(w, i));
}
template <int K>
__device__ __forceinline__ void obj_hits(const Ws &w, int t, int *h) {
  if constexpr (K == 3) {
    const int4 abc = gload(w.t3_md, t);
    const int md[3] = {abc.x, abc.y, abc.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int2 hh = w.md_hits[md[k]];
      h[2 * k] = hh.x;
      h[2 * k + 1] = hh.y;
    }
  } else {
    t5_hits(w, t, h);
  }
}

// pT duplicate removal: dropped when another entry with the same seed or the
// same outer object has a smaller (score, seed, hit tuple).  Entries of one
// seed differ in their outer object, so of a seed's entries only the one
// with the smallest (score, hit tuple) can survive; one wave per seed finds
// it (a minimum over the seed's entries, the hit tuples compared only on an
// exact tie of scores) and checks it alone against the entries sharing its
// outer object, whose tuples differ from it in the seed only: it survives if
// it has the object's smallest (score, seed) (k_pt_obj_best).
template <int K>
__global__ void k_pt_dedup(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = K == 3 ? w.ctr[C_NPT3] : w.ctr[C_NPT5];
  const int2 *so = K == 3 ? w.pt3_so : w.pt5_so;
  const float4 *at = K == 3 ? w.pt3_attr : w.pt5_attr;
  const int *soff = K == 3 ? w.pt3_off : w.pt5_off;
  const unsigned long long *obest = K == 3 ? w.o3_best : w.o5_best;
  int *keep = K == 3 ? w.pt3_keep : w.pt5_keep;
  constexpr int H = 2 * K + 1;
  const int lane = lane_id();
  const int wpb = blockDim.x >> 6;
  for (int s = blockIdx.x * wpb + (threadIdx.x >> 6); s < w.n_seeds; s += gridDim.x * wpb) {
    const int j0 = min(soff[s], n), j1 = min(soff[s + 1], n);
    if (j0 >= j1) continue;
    // the smallest score of the seed's entries (scores of accepted entries are finite)
    float best = 3.0e38f;
    for (int j = j0 + lane; j < j1; j += 64) best = fminf(best, at[j].z);
    for (int o = 32; o > 0; o >>= 1) best = fminf(best, __shfl_xor(best, o, 64));
    // the entry of that score with the smallest hit tuple (every lane scans the ties in order)
    int win = -1;
    int tw[H];
    for (int c0 = j0; c0 < j1; c0 += 64) {
      const int j = c0 + lane;
      const bool tie = j < j1 && !(best < at[j].z) && !(at[j].z < best);
      unsigned long long m = __ballot(tie);
      while (m) {
        const int l = __builtin_ctzll(m);
        m &= m - 1;
        const int jt = c0 + l;
        int tj[H];
        tj[0] = s;
        obj_hits<K>(w, so[jt].y, tj + 1);
        if (win < 0 || better<H>(best, tj, best, tw)) {
          win = jt;
#pragma unroll
          for (int q = 0; q < H; ++q) tw[q] = tj[q];
        }
      }
    }
    if (win < 0) {  // no finite score (not produced by the selection): keep none
      for (int j = j0 + lane; j < j1; j += 64) keep[j] = 0;
      continue;
    }
    // the winner survives the same-object rule if it is its object's best (score, seed)
    const bool kp = obest[so[win].y] == pt_obj_key<K>(w, win);
    for (int j = j0 + lane; j < j1; j += 64) keep[j] = (j == win && kp) ? 1 : 0;
  }
}

// ------------------------------------------------------------- a8: TC
__device__ __forceinline__ Dir dir_of_seed(const Ws &w, int s) { return seed_dir(load_seed(w, s)); }
__device__ __forceinline__ Dir dir_of_t5(const Ws &w, int t) {
  const float *a = w.t5_attr + 8 * (long)t;
  Dir d;
  d.dx = a[6]; d.dy = a[7]; d.lam = a[3];
  return d;
}

// pT5 TCs: every surviving pT5; marks its seed and T5 as used.
__global__ void k_tc_pt5(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = uload(w.ctr + C_NPT5);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int k = w.pt5_keep[i];
    w.f_pt5[i] = k;
    if (k) {
      w.seed_used[gload(w.pt5_so, i).x] = 1;
      w.t5_used[gload(w.pt5_so, i).y] = 1;
    }
  }
}
__global__ void k_tc_dirs_pt5(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = uload(w.ctr + C_NPT5);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    if (w.f_pt5[i]) {
      const Dir d = dir_of_seed(w, gload(w.pt5_so, i).x);
      w.dir_pt5[w.p_pt5[i]] = make_float4(d.dx, d.dy, d.lam, 0.f);
    }
}

// Direction lists of track candidates are binned by azimuth so that a
// proximity query reads only the bins that can hold a near entry.  Near
// entries have |dphi| < asin(D) (the test requires sin^2 dphi < D^2 and a
// positive dot product), so with bins of width 2 pi / kDirBins the query
// covers ceil(asin(D) / width) + 1 bins on each side, one more than needed
// to absorb atan2f rounding.  The decision itself is near_dir, unchanged.
constexpr int kDirBins = 128;

__device__ __forceinline__ int dir_bin(float dx, float dy) {
  const float ph = atan2f(dy, dx);
  if (!(ph == ph)) return 0;
  const int b = (int)floorf((ph + (float)M_PI) * (float)(kDirBins / (2.0 * M_PI)));
  return b < 0 ? 0 : (b >= kDirBins ? kDirBins - 1 : b);
}

constexpr int bin_reach(double D) {
  // ceil(asin(D) / (2 pi / kDirBins)) + 1 for the D values used (asin(D) < 1.0001 D for D <= 0.05)
  return (int)(D * 1.0001 / (2.0 * 3.14159265358979 / kDirBins)) + 2;
}

// One block: counting sort of n (on the device) directions into kDirBins bins.
__global__ __launch_bounds__(1024) void k_bin_dirs(const Ws *__restrict__ wb, int which) {
  __shared__ int s_cnt[kDirBins], s_off[kDirBins + 1], s_cur[kDirBins];
  const Ws &w = wb[blockIdx.y];
  const float4 *dirs = which == 0 ? w.dir_pt5 : (which == 1 ? w.dir_pt3 : w.dir_t5);
  int *bin_off = which == 0 ? w.boff_pt5 : (which == 1 ? w.boff_pt3 : w.boff_t5);
  float4 *out = which == 0 ? w.bdir_pt5 : (which == 1 ? w.bdir_pt3 : w.bdir_t5);
  const int n = w.ctr[which == 0 ? C_NTC0 : (which == 1 ? C_NTC1 : C_NTC2)];
  for (int b = threadIdx.x; b < kDirBins; b += blockDim.x) { s_cnt[b] = 0; s_cur[b] = 0; }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) atomicAdd(&s_cnt[dir_bin(dirs[i].x, dirs[i].y)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int r = 0;
    for (int b = 0; b < kDirBins; ++b) { s_off[b] = r; r += s_cnt[b]; }
    s_off[kDirBins] = r;
  }
  __syncthreads();
  for (int b = threadIdx.x; b <= kDirBins; b += blockDim.x) bin_off[b] = s_off[b];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float4 d = dirs[i];
    const int b = dir_bin(d.x, d.y);
    out[s_off[b] + atomicAdd(&s_cur[b], 1)] = d;
  }
}

// Wave-cooperative query: the 64 lanes stride over the entries of the bins
// around the query's azimuth; returns (to every lane) whether any is near.
// `d` and `active` must be wave-uniform.
__device__ __forceinline__ bool near_any_wave(const Dir &d, bool active, const float4 *lst, const int *bin_off, float D,
                                              int reach) {
  if (!active) return false;
  const int lane = lane_id();
  const int b0 = dir_bin(d.dx, d.dy);
  for (int k = -reach; k <= reach; ++k) {
    const int b = (b0 + k + kDirBins) % kDirBins;
    const int j0 = bin_off[b], j1 = bin_off[b + 1];
    for (int j = j0 + lane; j - lane < j1; j += 64) {
      bool nr = false;
      if (j < j1) {
        const float4 e = lst[j];
        Dir o;
        o.dx = e.x; o.dy = e.y; o.lam = e.z;
        nr = near_dir(d, o, D);
      }
      if (__ballot(nr)) return true;
    }
  }
  return false;
}

// pT3 TCs: surviving pT3 whose seed no TC-pT5 uses and that is not near any TC-pT5.
// One wave per candidate (the query loops over binned lists with its lanes).
__global__ void k_tc_pt3(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = uload(w.ctr + C_NPT3);
  const int wpb = blockDim.x >> 6;
  const int nw = gridDim.x * wpb;
  for (int i = blockIdx.x * wpb + (threadIdx.x >> 6); i < n; i += nw) {
    const int s = gload(w.pt3_so, i).x;
    const bool cand = w.pt3_keep[i] && !w.seed_used[s];
    const bool nr = near_any_wave(dir_of_seed(w, s), cand, w.bdir_pt5, w.boff_pt5, kDpT3, bin_reach(0.02));
    if (lane_id() == 0) w.f_pt3[i] = (cand && !nr) ? 1 : 0;
  }
}
__global__ void k_tc_dirs_pt3(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = uload(w.ctr + C_NPT3);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    if (w.f_pt3[i]) {
      const int s = gload(w.pt3_so, i).x;
      const Dir d = dir_of_seed(w, s);
      w.dir_pt3[w.p_pt3[i]] = make_float4(d.dx, d.dy, d.lam, 0.f);
      w.seed_used[s] = 1;
    }
}
// T5 TCs: surviving T5 not used by a TC-pT5 and not near any TC-pT5 or TC-pT3.
__global__ void k_tc_t5(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = uload(w.ctr + C_NT5);
  const int wpb = blockDim.x >> 6;
  const int nw = gridDim.x * wpb;
  for (int t = blockIdx.x * wpb + (threadIdx.x >> 6); t < n; t += nw) {
    const bool cand = gp(w.t5_keep)[t] && !w.t5_used[t];
    const Dir d = dir_of_t5(w, t);
    const bool nr = near_any_wave(d, cand, w.bdir_pt5, w.boff_pt5, kDT5, bin_reach(0.02)) ||
                    near_any_wave(d, cand, w.bdir_pt3, w.boff_pt3, kDT5, bin_reach(0.02));
    if (lane_id() == 0) w.f_t5[t] = (cand && !nr) ? 1 : 0;
  }
}
__global__ void k_tc_dirs_t5(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = uload(w.ctr + C_NT5);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
    if (w.f_t5[t]) {
      const Dir d = dir_of_t5(w, t);
      w.dir_t5[w.p_t5[t]] = make_float4(d.dx, d.dy, d.lam, 0.f);
    }
}
// pLS TCs: surviving pLS used by no TC and not near any TC.
__global__ void k_tc_pls(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int wpb = blockDim.x >> 6;
  const int nw = gridDim.x * wpb;
  for (int s = blockIdx.x * wpb + (threadIdx.x >> 6); s < w.n_seeds; s += nw) {
    const bool cand = gp(w.pls_keep)[s] && !w.seed_used[s];
    const Dir d = dir_of_seed(w, s);
    const bool nr = near_any_wave(d, cand, w.bdir_pt5, w.boff_pt5, kDpLS, bin_reach(0.05)) ||
                    near_any_wave(d, cand, w.bdir_pt3, w.boff_pt3, kDpLS, bin_reach(0.05)) ||
                    near_any_wave(d, cand, w.bdir_t5, w.boff_t5, kDpLS, bin_reach(0.05));
    if (lane_id() == 0) w.f_pls[s] = (cand && !nr) ? 1 : 0;
  }
}

// What the track-extension step reads of a candidate: its MDs and its
// curvature with tolerance (the seed's, three resolutions, for pT5 / pT3;
// the five-anchor fit's and the outer triplet's resolution for a T5).
__device__ __forceinline__ float2 seed_kappa(const Ws &w, int seed) {
  const float ks = gp(w.pls)[8 * (long)seed + 4];
  return make_float2(ks, 3.0f * (kSeedDpt * fabsf(ks)));
}
__device__ __forceinline__ void ext_record(const Ws &w, int k, const int *md, int K, float2 kap) {
  for (int i = 0; i < K; ++i) w.tc_md[5 * (long)k + i] = md[i];
  gstore(w.tc_kap, k, kap);
}

// Output: type, offsets, hit lists (pixel hits first, then MD hits inner to outer).
__global__ void k_tc_write(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n0 = uload(w.ctr + C_NTC0), n1 = uload(w.ctr + C_NTC1), n2 = uload(w.ctr + C_NTC2), n3 = uload(w.ctr + C_NTC3);
  const int np5 = uload(w.ctr + C_NPT5), np3 = uload(w.ctr + C_NPT3), nt5 = uload(w.ctr + C_NT5);
  const long h1 = 14L * n0, h2 = h1 + 10L * n1, h3 = h2 + 10L * n2;
  const int stride = gridDim.x * blockDim.x;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0) {
    w.ctr[C_NTC] = n0 + n1 + n2 + n3;
    w.ctr[C_NTCHITS] = (int)(h3 + 4L * n3);
    w.tc_off[n0 + n1 + n2 + n3] = (int)(h3 + 4L * n3);
  }
  for (int i = tid; i < np5; i += stride) {
    if (!w.f_pt5[i]) continue;
    const int k = w.p_pt5[i];
    const int2 so = gload(w.pt5_so, i);
    int *h = w.tc_hits + 14L * k;
    for (int q = 0; q < 4; ++q) h[q] = gp(w.hits4)[4 * (long)so.x + q];
    t5_hits(w, so.y, h + 4);
    w.tc_type[k] = 0;
    ext_record(w, k, w.t5_md + 5 * (long)so.y, 5, seed_kappa(w, so.x));
    w.tc_off[k] = 14 * k;
  }
  for (int i = tid; i < np3; i += stride) {
    if (!w.f_pt3[i]) continue;
    const int k = w.p_pt3[i];
    const int2 so = gload(w.pt3_so, i);
    int *h = w.tc_hits + h1 + 10L * k;
    for (int q = 0; q < 4; ++q) h[q] = gp(w.hits4)[4 * (long)so.x + q];
    obj_hits<3>(w, so.y, h + 4);
    w.tc_type[n0 + k] = 1;
    {
      const int4 abc = gload(w.t3_md, so.y);
      const int md[3] = {abc.x, abc.y, abc.z};
      ext_record(w, n0 + k, md, 3, seed_kappa(w, so.x));
    }
    w.tc_off[n0 + k] = (int)(h1 + 10L * k);
  }
  for (int t = tid; t < nt5; t += stride) {
    if (!w.f_t5[t]) continue;
    const int k = w.p_t5[t];
    t5_hits(w, t, w.tc_hits + h2 + 10L * k);
    w.tc_type[n0 + n1 + k] = 2;
    ext_record(w, n0 + n1 + k, w.t5_md + 5 * (long)t, 5,
               make_float2(w.t5_attr[8 * (long)t], w.t3_attr[gload(w.t5_t3, t).y].y));
    w.tc_off[n0 + n1 + k] = (int)(h2 + 10L * k);
  }
  for (int s = tid; s < w.n_seeds; s += stride) {
    if (!w.f_pls[s]) continue;
    const int k = w.p_pls[s];
    int *h = w.tc_hits + h3 + 4L * k;
    for (int q = 0; q < 4; ++q) h[q] = gp(w.hits4)[4 * (long)s + q];
    w.tc_type[n0 + n1 + n2 + k] = 3;
    w.tc_off[n0 + n1 + n2 + k] = (int)(h3 + 4L * k);
  }
}

// ------------------------------------------------- track extensions (S2.5)
// A candidate with outer MDs (pT5, pT3, T5) is tested against the triplets
// whose first two MDs are its last two (one MD added) and those whose first
// MD is its last (two added): curvatures within their resolutions (the
// seed's for pT5 / pT3, three resolutions; the outer triplet's for a T5),
// azimuth linear in z over the first, the candidate's last and the last
// added anchor, and the widened quintuplet fits (ext_fit).  The passing
// triplet adding more MDs wins, then the smaller chi2_xy + chi2_rz, then the
// smaller hit tuple of the added MDs.
//
// A wave takes kExtPerWave candidates; their (candidate, triplet) pairs are
// laid out flat (wave_segments) so the lanes test one pair each, and every
// candidate's lane then merges the passing pairs of its segment from LDS.  (A thread per
// candidate walking its own triplets is bound by the longest such walk.)
// (add, score, hits) of a strictly better than those of b
__device__ __forceinline__ bool ext_better(int add_a, float sc_a, int4 h_a, int add_b, float sc_b, int4 h_b) {
  if (add_a != add_b) return add_a > add_b;
  if (sc_a < sc_b) return true;
  if (sc_b < sc_a) return false;
  const int ha[4] = {h_a.x, h_a.y, h_a.z, h_a.w}, hb[4] = {h_b.x, h_b.y, h_b.z, h_b.w};
  for (int i = 0; i < 2 * add_a; ++i)
    if (ha[i] != hb[i]) return ha[i] < hb[i];
  return false;
}

// The K anchors of a candidate (K = 3 or 5; sP / sM [0..K)[e], staged in
// LDS) followed by the ADD MDs of triplet abc in the kExtMax slots of ext_fit
// (the slots past the chain repeat its last anchor), tested with the
// lever-arm azimuth-z check and ext_fit; the added MDs' hits come back in h.
template <int C>
__device__ __forceinline__ bool ext_eval(const Ws &w, const DevGeom &g, const float4 (*sP)[C], const int (*sM)[C],
                                         int e, int K, int add, int4 abc, float3 *a, int4 *h) {
  const int nm0 = add == 1 ? abc.z : abc.y;
  const float4 A0 = gload(w.md_pos, nm0);
  const int mod0 = gp(w.md_mod)[nm0];
  const int2 h0 = gload(w.md_hits, nm0);
  float4 A1 = A0;
  int mod1 = mod0;
  int2 h1 = make_int2(0, 0);
  if (add == 2) {
    A1 = gload(w.md_pos, abc.z);
    mod1 = gp(w.md_mod)[abc.z];
    h1 = gload(w.md_hits, abc.z);
  }
  ModInfo I0, I1;
  I0.bits = gp(g.info)[mod0];
  I1.bits = gp(g.info)[mod1];
  float4 P[kExtMax];
  ModInfo M[kExtMax];
#pragma unroll
  for (int i = 0; i < kExtMax; ++i) {
    if (i < 5 && i < K) {
      P[i] = sP[i][e];
      M[i].bits = sM[i][e];
    } else {
      P[i] = i == K ? A0 : A1;
      M[i] = i == K ? I0 : I1;
    }
  }
  *h = make_int4(h0.x, h0.y, h1.x, h1.y);
  const float4 PK = K == 5 ? P[4] : P[2];
  const ModInfo MK = K == 5 ? M[4] : M[2];
  return phiz_pass(P[0], PK, A1, M[0], MK, I1, g.d0max) && ext_fit(P, M, K + add, a);
}

// Candidates per wave, C (tile ext_per_wave: 4, 8 or 16): few enough that
// their (candidate, triplet) pairs (about 1.3 per candidate) spread over many
// waves.
template <int C>
__global__ __launch_bounds__(kBlock) void k_tc_ext(const Ws *__restrict__ wb, DevGeom g) {
  const Ws &w = wb[blockIdx.y];
  constexpr int kExtPerWave = C;
  __shared__ float4 s_P[kWaves][5][C];  // the candidates' anchors
  __shared__ int s_M[kWaves][5][C], s_md[kWaves][C], s_k[kWaves][C], s_lo2[kWaves][C], s_n2[kWaves][C],
      s_lo1[kWaves][C];  // module info bits, last MD, MD count, triplet ranges
  __shared__ int s_seg[kWaves][65];
  __shared__ float s_kt[kWaves][C], s_dkt[kWaves][C];
  __shared__ int s_rt[kWaves][64], s_radd[kWaves][64];  // per pair of the round: triplet (-1: fails), MDs added
  __shared__ float s_rsc[kWaves][64];
  __shared__ int4 s_rh[kWaves][64];
  __shared__ float4 s_ra[kWaves][64];
  const int n = uload(w.ctr + C_NTC);
  const int n_ls = uload(w.ctr + C_NLS), n_t3 = uload(w.ctr + C_NT3);
  const int wv = wave_id(), lane = lane_id();
  const int wpb = blockDim.x >> 6;
  for (long p0 = ((long)blockIdx.x * wpb + wv) * kExtPerWave; p0 < n; p0 += (long)gridDim.x * wpb * kExtPerWave) {
    const int k = (int)p0 + lane;
    const bool mine = lane < kExtPerWave && k < n;
    int cnt = 0;
    if (mine) {
      const int type = w.tc_type[k];
      const int K = type == 3 ? 0 : (type == 1 ? 3 : 5);
      s_k[wv][lane] = K;
      if (K > 0) {
        int md[5];
#pragma unroll
        for (int i = 0; i < 5; ++i) md[i] = i < K ? w.tc_md[5 * (long)k + i] : 0;
        const float2 kap = gload(w.tc_kap, k);
        s_kt[wv][lane] = kap.x;
        s_dkt[wv][lane] = kap.y;
#pragma unroll
        for (int i = 0; i < 5; ++i)
          if (i < K) {
            s_P[wv][i][lane] = w.md_pos[md[i]];
            s_M[wv][i][lane] = gp(g.info)[gp(w.md_mod)[md[i]]];
          }
        // triplets with first MD m: those built from segments with inner MD m
        const int m2 = K == 5 ? md[3] : md[1], m1 = K == 5 ? md[4] : md[2];
        s_md[wv][lane] = m1;
        const int l2b = min(w.ls_off[m2], n_ls), l2e = min(w.ls_off[m2 + 1], n_ls);
        const int l1b = min(w.ls_off[m1], n_ls), l1e = min(w.ls_off[m1 + 1], n_ls);
        const int lo2 = gp(w.t3_off)[l2b], hi2 = min(w.t3_off[l2e], n_t3);
        const int lo1 = gp(w.t3_off)[l1b], hi1 = min(w.t3_off[l1e], n_t3);
        const int n2 = hi2 > lo2 ? hi2 - lo2 : 0, n1 = hi1 > lo1 ? hi1 - lo1 : 0;
        s_lo2[wv][lane] = lo2;
        s_n2[wv][lane] = n2;
        s_lo1[wv][lane] = lo1;
        cnt = n2 + n1;
      }
    }
    const int total = wave_segments(cnt, s_seg[wv]);
    int best_n = 0, best_t = -1;
    float best_s = 0.0f;
    int4 best_h = make_int4(0, 0, 0, 0);
    float4 best_a = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    int e = 0;  // candidate of this lane's pair (pairs advance monotonically)
    for (int c0 = 0; c0 < total; c0 += 64) {
      const int c = c0 + lane;
      int rt = -1, radd = 0;
      float rsc = 0.0f;
      int4 rh = make_int4(0, 0, 0, 0);
      float4 ra = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (c < total) {
        while (s_seg[wv][e + 1] <= c) ++e;
        const int idx = c - s_seg[wv][e];
        const int K = s_k[wv][e], n2 = s_n2[wv][e];
        const int ov = idx < n2 ? 2 : 1;
        const int t = ov == 2 ? s_lo2[wv][e] + idx : s_lo1[wv][e] + (idx - n2);
        const int4 abc = gload(w.t3_md, t);
        const float4 ta = gload(w.t3_attr, t);
        const int add = 3 - ov;
        const float dk = ta.x - s_kt[wv][e];
        bool ok = ov == 1 || abc.y == s_md[wv][e];
        ok = ok && fabsf(dk) <= ta.y + s_dkt[wv][e];
        if (ok) {
          // the anchors fill ext_fit's fixed slots (static indices: they stay in registers)
          float3 a;
          int4 h;
          if (ext_eval(w, g, s_P[wv], s_M[wv], e, K, add, abc, &a, &h)) {
            rt = t;
            radd = add;
            rsc = a.x + a.y;
            rh = h;
            ra = make_float4(a.x, a.y, a.z, 0.0f);
          }
        }
      }
      s_rt[wv][lane] = rt;
      s_radd[wv][lane] = radd;
      s_rsc[wv][lane] = rsc;
      s_rh[wv][lane] = rh;
      s_ra[wv][lane] = ra;
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // every candidate merges the pairs of its segment that fell in this round
      const int q0 = max(s_seg[wv][lane], c0) - c0, q1 = min(s_seg[wv][lane + 1], c0 + 64) - c0;
      for (int q = q0; q < q1; ++q) {
        const int t = s_rt[wv][q];
        if (t < 0) continue;
        const int add = s_radd[wv][q];
        const float sc = s_rsc[wv][q];
        const int4 h = s_rh[wv][q];
        if (best_t < 0 || ext_better(add, sc, h, best_n, best_s, best_h)) {
          best_n = add; best_t = t; best_s = sc; best_h = h; best_a = s_ra[wv][q];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
    if (mine) {
      w.ext_n[k] = best_n;
      w.ext_t3[k] = best_t;
      gstore(w.ext_attr, k, best_a);
      w.ext_cnt[k] = (w.tc_off[k + 1] - w.tc_off[k]) + 2 * best_n;
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// The extended collection: each candidate's hits, then those of its added MDs.
__global__ void k_tc_ext_write(const Ws *__restrict__ wb) {
  const Ws &w = wb[blockIdx.y];
  const int n = uload(w.ctr + C_NTC);
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  if (tid == 0) w.ctr[C_EXT] = 1;
  for (int k = tid; k < n; k += gridDim.x * blockDim.x) {
    int *dst = w.ext_hits + w.ext_off[k];
    const int b1 = w.tc_off[k + 1];
    for (int h = w.tc_off[k]; h < b1; ++h) *dst++ = w.tc_hits[h];
    const int na = w.ext_n[k];
    if (na > 0) {
      const int4 abc = w.t3_md[w.ext_t3[k]];
      int2 hh = gload(w.md_hits, na == 1 ? abc.z : abc.y);
      dst[0] = hh.x;
      dst[1] = hh.y;
      if (na == 2) {
        hh = gload(w.md_hits, abc.z);
        dst[2] = hh.x;
        dst[3] = hh.y;
      }
    }
  }
}

// ------------------------------------------------------------- chain
// Launch sites of the chain, in order; each is launched once per event.  One
// of them can be bracketed by HIP events (KernelTimer) to time it live.
const char *const kSiteNames[] = {
    "fill_counters", "hits_count", "hits_scan", "hits_scatter", "bucket_sort",
    "md_count", "md_scan", "md_fill", "ls_count", "ls_scan", "ls_fill",
    "t3_count", "t3_scan", "t3_fill", "t5_count", "t5_scan", "t5_fill",
    "t5_inc_count", "t5_inc_scan", "t5_inc_scatter", "t5_dedup",
    "pls", "pls_hit_scan", "pls_hit_scatter", "pls_dedup",
    "pt3_bin", "pt5_bin", "pt_count", "pt3_scan", "pt3_fill", "pt5_scan", "pt5_fill",
    "pt_obj_best", "pt3_dedup", "pt5_dedup",
    "tc_pt5", "tc_pt5_scan", "tc_pt5_dirs", "tc_pt3", "tc_pt3_scan", "tc_pt3_dirs",
    "tc_t5", "tc_t5_scan", "tc_t5_dirs", "tc_pls", "tc_pls_scan", "tc_write",
    "tc_ext", "tc_ext_scan", "tc_ext_write"};
const int kNumSites = (int)(sizeof(kSiteNames) / sizeof(kSiteNames[0]));
static_assert(sizeof(kSiteNames) / sizeof(kSiteNames[0]) <= kMaxSites, "launch-site table");

// Sites whose kernels take any block of 64, 128 or 256 threads (grid-stride
// loops over threads or waves, LDS sized for the largest block): the launch
// shape the autotuner may choose.
static const char *const kTunableSites[] = {"md_count", "md_fill",  "ls_count", "ls_fill",  "t3_count",
                                            "t3_fill",  "t5_count", "t5_fill",  "t5_dedup", "pt_count",
                                            "pt3_fill", "pt5_fill", "tc_pt3",   "tc_t5",    "tc_pls",
                                            "tc_ext"};

bool site_tunable(int site) {
  if (site < 0 || site >= kNumSites) return false;
  for (const char *n : kTunableSites)
    if (std::strcmp(n, kSiteNames[site]) == 0) return true;
  return false;
}

// Inner MDs per wave of the segment count pass: the tile when set, else
// enough groups for about 32k waves over the launch's events (MDs taken as a
// quarter of the MD capacity, which defaults to the hit count): one event
// alone gets groups of 4, launches of 16 or more PU200-size events groups of 16.
int ls_group_for(const Tiles &t, int B, long cap_md) {
  if (t.ls_group > 0) return t.ls_group < kLsGroup ? t.ls_group : kLsGroup;
  const long gsz = (long)B * (cap_md / 4) / 32768;
  return (int)std::max(1L, std::min((long)kLsGroup, gsz));
}

void enqueue_chain(const DevGeom &g, const Ws *wb, int B, const Ws &b, hipStream_t st, const KernelTimer *kt,
                   const int *site_block) {
  int site = 0;
  int tb = kBlock;  // block size of the current site (tunable sites only)
  // Runs one launch site; the timed site is bracketed by the timer's events.
  auto run = [&](auto &&launch) {
    const bool timed = kt && kt->site == site;
    tb = (site_block && site_block[site] > 0) ? site_block[site] : kBlock;
    if (timed) (void)hipEventRecord(kt->beg, st);
    launch();
    if (timed) (void)hipEventRecord(kt->end, st);
    ++site;
  };
  const int M = g.n_mod;
  const long N = b.n_hits, S = b.n_seeds;  // largest of the batch
  const bool seeds = S > 0;
  // Blocks per event: what the capacity would ask for, but at most an equal share of
  // kLaunchWaves.  The kernels launched through these stride over their device-side
  // counts, and the counts are far below the capacities: a launch over many events
  // would otherwise spend most of its time dispatching blocks that find no work.
  const long ev_waves = std::max(256L, kLaunchWaves / B);
  auto share = [&](int blocks, int threads) {
    return (unsigned)std::max(1L, std::min((long)blocks, ev_waves / (threads / 64)));
  };
  auto share_big = [&](int blocks, int threads) {
    return (unsigned)std::max(1L, std::min((long)blocks, 4 * ev_waves / (threads / 64)));
  };
  auto grid = [&](long n) { return dim3(share(grid_for(n), kBlock), B); };
  auto gridt = [&](long n) { return dim3(share(grid_for(n, tb), tb), B); };    // tuned thread-per-item sites
  auto gridwt = [&](long n) { return dim3(share(grid_waves(n, tb), tb), B); }; // tuned wave-per-item sites
  auto gridwb = [&](long n) { return dim3(share_big(grid_waves(n, tb), tb), B); }; // the heavy searches
  // one wave per seed, every seed its own wave (the seed search does not stride)
  auto seedwaves = [&] { return dim3((unsigned)((S + tb / 64 - 1) / (tb / 64) > 0 ? (S + tb / 64 - 1) / (tb / 64) : 1), B); };
  const dim3 one(1, B);
  const bool whole = kt && kt->site == kChainSite;  // the timer brackets the whole chain
  if (whole) (void)hipEventRecord(kt->beg, st);
  // a0: buckets
  run([&] { k_clear<<<grid(C_COUNT), kBlock, 0, st>>>(wb, FL_CTR, FL_CTR + 1); });
  const long n_tiles = n_hit_tiles(N), n_co = n_coarse(M);
  run([&] {  // one block per hit tile, and enough threads for the seeds' validation
    const long blocks = std::max(n_tiles, (S + kBlock - 1) / kBlock);
    k_hits_count<<<dim3((unsigned)std::max(1L, std::min(blocks, 65535L)), B), kBlock, kWaves * n_co * sizeof(int), st>>>(wb, M);
  });
  run([&] { scan(wb, B, SC_HITS, n_co * n_tiles, st); });
  run([&] { k_hits_scatter<<<dim3((unsigned)std::max(1L, n_tiles), B), kBlock, kWaves * n_co * sizeof(int), st>>>(wb, M); });
  run([&] { k_bucket_sort<<<dim3((unsigned)n_co, B), 64 * kSortWaves, 0, st>>>(wb, M); });
  // a1: MD (a dense module's block: kMdParts waves for a launch of one event, else 4)
  const int md_big_threads = 64 * (B == 1 ? kMdParts : 4);
  run([&] {  // the small modules' count lists the dense ones for k_md_big
    k_md<false><<<gridwb(M), tb, 0, st>>>(wb, g);
    k_md_big<false><<<dim3(share(1024, md_big_threads), B), md_big_threads, 0, st>>>(wb, g);
  });
  run([&] { scan(wb, B, SC_MD, M, st); });
  run([&] {
    k_md_big<true><<<dim3(share(1024, md_big_threads), B), md_big_threads, 0, st>>>(wb, g);
    k_md<true><<<gridwb(M), tb, 0, st>>>(wb, g);
  });
  // a2: LS
  run([&] {
    const int lg = ls_group_for(g.tiles, B, b.cap_md);
    k_ls_count<<<gridwb((b.cap_md + lg - 1) / lg), tb, 0, st>>>(wb, g, lg);
  });
  run([&] { scan(wb, B, SC_LS, b.cap_md, st); });
  run([&] {
    scan(wb, B, SC_LSOVF, b.cap_md, st);
    k_ls_copy<<<gridt((long)b.cap_md * kLsCopyLanes), tb, 0, st>>>(wb, g.tiles.ls_cache);
    k_ls_fill<<<gridwt(b.cap_md < 16384 ? b.cap_md : 16384), tb, 0, st>>>(wb, g);  // the overflow MDs
  });
  // a3: T3
  run([&] { k_t3<false><<<gridwb((b.cap_ls + 63) / 64), tb, 0, st>>>(wb, g); });
  run([&] { scan(wb, B, SC_T3, b.cap_ls, st); });
  run([&] { k_t3<true><<<gridwb((b.cap_ls + 63) / 64), tb, 0, st>>>(wb, g); });
  // a4: T5
  run([&] { k_t5<false><<<gridwb((b.cap_t3 + 63) / 64), tb, 0, st>>>(wb, g); });
  run([&] { scan(wb, B, SC_T5, b.cap_t3, st); });
  run([&] { k_t5<true><<<gridwb((b.cap_t3 + 63) / 64), tb, 0, st>>>(wb, g); });
  // a5: T5 duplicate removal through per-MD incidence lists
  run([&] {
    k_clear<<<grid((long)b.cap_md + 1), kBlock, 0, st>>>(wb, FL_INC_CNT, FL_INC_CUR + 1);
    k_t5_inc_count<<<grid(b.cap_t5), kBlock, 0, st>>>(wb);
  });
  run([&] { scan(wb, B, SC_INC, b.cap_md, st); });
  run([&] { k_t5_inc_scatter<<<grid(b.cap_t5), kBlock, 0, st>>>(wb); });
  run([&] {
    const int ipw = B == 1 ? 16 : 64;
    k_t5_dedup<<<gridwb((4L * b.cap_t5 + ipw - 1) / ipw), tb, (tb / 64) * kT5DedupLds, st>>>(wb, ipw);
  });
  // a6: pLS
  run([&] {
    k_clear<<<grid(N + 1), kBlock, 0, st>>>(wb, FL_PH_CNT, FL_PH_CUR + 1);
    if (seeds) k_pls<<<grid(S), kBlock, 0, st>>>(wb);
  });
  run([&] { if (seeds) scan(wb, B, SC_PH, N, st); });
  run([&] { if (seeds) k_ph_scatter<<<grid(S), kBlock, 0, st>>>(wb); });
  run([&] { if (seeds) k_pls_dedup<<<grid(S), kBlock, 0, st>>>(wb); });
  // a7: pT3, pT5: objects binned by first anchor, one wave per seed over its bins
  run([&] {
    if (!seeds) return;
    k_clear<<<grid(kSeedBins + 1), kBlock, 0, st>>>(wb, FL_B3_CNT, FL_B5_CUR + 1);
    k_seed_order<<<one, 1024, 0, st>>>(wb);
    k_obj_bin_count<3><<<grid(b.cap_t3), kBlock, 0, st>>>(wb);
    scan(wb, B, SC_B3, kSeedBins, st);
    k_obj_bin_scatter<3><<<grid(b.cap_t3), kBlock, 0, st>>>(wb, g);
  });
  run([&] {
    if (!seeds) return;
    k_obj_bin_count<5><<<grid(b.cap_t5), kBlock, 0, st>>>(wb);
    scan(wb, B, SC_B5, kSeedBins, st);
    k_obj_bin_scatter<5><<<grid(b.cap_t5), kBlock, 0, st>>>(wb, g);
  });
  // both counts on one trajectory mask per seed
  run([&] { if (seeds) k_pt_binned<3, false, true><<<seedwaves(), tb, 0, st>>>(wb, g); });
  run([&] { if (seeds) scan(wb, B, SC_PT3, S, st); });
  run([&] { if (seeds) k_pt_binned<3, true><<<seedwaves(), tb, 0, st>>>(wb, g); });
  run([&] { if (seeds) scan(wb, B, SC_PT5, S, st); });
  run([&] { if (seeds) k_pt_binned<5, true><<<seedwaves(), tb, 0, st>>>(wb, g); });
  run([&] {
    if (!seeds) return;
    const long n = 2L * ((b.cap_t3 > b.cap_t5 ? b.cap_t3 : b.cap_t5) + 1);
    k_clear<<<grid(n), kBlock, 0, st>>>(wb, FL_O3_BEST, FL_O5_BEST + 1);
    k_pt_obj_best<3><<<grid(b.cap_pt3), kBlock, 0, st>>>(wb);
    k_pt_obj_best<5><<<grid(b.cap_pt5), kBlock, 0, st>>>(wb);
  });
  run([&] { if (seeds) k_pt_dedup<3><<<dim3(grid_waves(S), B), kBlock, 0, st>>>(wb); });
  run([&] { if (seeds) k_pt_dedup<5><<<dim3(grid_waves(S), B), kBlock, 0, st>>>(wb); });
  // a8: cleaning and track candidates
  run([&] {
    const long n = (long)(S > b.cap_t5 ? S : b.cap_t5) + 1;
    k_clear<<<grid(n), kBlock, 0, st>>>(wb, FL_SEED_USED, FL_T5_USED + 1);
    k_tc_pt5<<<grid(b.cap_pt5), kBlock, 0, st>>>(wb);
  });
  run([&] { scan(wb, B, SC_F5, b.cap_pt5, st); });
  run([&] {
    k_tc_dirs_pt5<<<grid(b.cap_pt5), kBlock, 0, st>>>(wb);
    k_bin_dirs<<<one, 1024, 0, st>>>(wb, 0);
  });
  run([&] { k_tc_pt3<<<gridwt(b.cap_pt3), tb, 0, st>>>(wb); });
  run([&] { scan(wb, B, SC_F3, b.cap_pt3, st); });
  run([&] {
    k_tc_dirs_pt3<<<grid(b.cap_pt3), kBlock, 0, st>>>(wb);
    k_bin_dirs<<<one, 1024, 0, st>>>(wb, 1);
  });
  run([&] { k_tc_t5<<<gridwt(b.cap_t5), tb, 0, st>>>(wb); });
  run([&] { scan(wb, B, SC_FT5, b.cap_t5, st); });
  run([&] {
    k_tc_dirs_t5<<<grid(b.cap_t5), kBlock, 0, st>>>(wb);
    k_bin_dirs<<<one, 1024, 0, st>>>(wb, 2);
  });
  run([&] { if (seeds) k_tc_pls<<<gridwt(S), tb, 0, st>>>(wb); });
  run([&] { if (seeds) scan(wb, B, SC_FPLS, S, st); });
  run([&] { k_tc_write<<<grid(b.cap_tc), kBlock, 0, st>>>(wb); });
  // track extensions (when the geometry enables them)
  run([&] {
    if (!g.ext) return;
    const int c = g.tiles.ext_per_wave;
    if (c == 4) k_tc_ext<4><<<gridwt((b.cap_tc + 3) / 4), tb, 0, st>>>(wb, g);
    else if (c == 16) k_tc_ext<16><<<gridwt((b.cap_tc + 15) / 16), tb, 0, st>>>(wb, g);
    else k_tc_ext<8><<<gridwt((b.cap_tc + 7) / 8), tb, 0, st>>>(wb, g);
  });
  run([&] { if (g.ext) scan(wb, B, SC_EXT, b.cap_tc, st); });
  run([&] { if (g.ext) k_tc_ext_write<<<grid(b.cap_tc), kBlock, 0, st>>>(wb); });
  if (whole) (void)hipEventRecord(kt->end, st);
}

}  // namespace lst
