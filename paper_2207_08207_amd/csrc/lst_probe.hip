// Calibration kernels for the counter summaries: kernels whose work is known
// exactly, against which the vector-issue counters of the chain's kernels are
// normalised (as a plain copy kernel calibrates the HBM byte counters).
#include <hip/hip_runtime.h>

#include "../../include/lst.h"

namespace {

// Every thread runs `iters` rounds of 16 independent fused multiply-adds
// (16 chains, so consecutive instructions never wait for each other): 16 VALU
// instructions per round and wave, plus the loop's few.  With enough waves per
// SIMD this is the issue rate of a SIMD that never stalls.
__global__ __launch_bounds__(256) void k_probe_valu(int iters, float *out) {
  float a[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) a[k] = (float)(threadIdx.x + k);
  const float m = 1.0000001f, c = 1e-7f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 16; ++k) a[k] = __builtin_fmaf(a[k], m, c);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += a[k];
  if (s == 123.0f) out[blockIdx.x * blockDim.x + threadIdx.x] = s;  // keeps the chains live
}

}  // namespace

extern "C" lst_status lst_probe_valu(int32_t n_blocks, int32_t iters, float *out, void *stream) {
  if (n_blocks < 1 || iters < 1 || !out) return LST_E_INVALID;
  k_probe_valu<<<n_blocks, 256, 0, reinterpret_cast<hipStream_t>(stream)>>>(iters, out);
  return hipGetLastError() == hipSuccess ? LST_OK : LST_E_DEVICE;
}
