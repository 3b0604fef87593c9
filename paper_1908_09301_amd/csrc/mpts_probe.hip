// Issue-rate probes of the two arithmetic units the Cauchy sums run on, for
// the roofline of the measurement: the VALU 32x32 -> 64-bit signed
// multiply-add (v_mad_i64_i32, the digit products of the tile path) and the
// int8 matrix-core instruction v_mfma_i32_32x32x32_i8 (the piece products of
// the matrix-core path).  Registers only: independent chains, no memory
// traffic inside the timed loop.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpts.h"

namespace {

// 8x8 digit tiles into 15 column sums, as the product loop forms them.
__global__ void __launch_bounds__(256) k_probe_mad(long long *out, int iters, int seed) {
  int u[8], v[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    u[r] = (int)(threadIdx.x * 2654435761u + r * 97u + seed) & 0x0fffffff;
    v[r] = (int)(threadIdx.x * 40503u + r * 31u - seed) & 0x0fffffff;
  }
  long long acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int s = 0; s < 8; ++s) acc[r + s] += (long long)u[r] * (long long)v[s];
    // keep the operands live and changing (one add per row, not timed work)
#pragma unroll
    for (int r = 0; r < 8; ++r) u[r] ^= it;
  }
  long long t = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) t += acc[r];
  out[blockIdx.x * blockDim.x + threadIdx.x] = t;
}

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

__global__ void __launch_bounds__(256) k_probe_mfma(long long *out, int iters, int seed) {
  v16i c0 = {}, c1 = {}, c2 = {}, c3 = {};
  const int l = threadIdx.x;
  v4i a = {1 + l + seed, 2, 3, 4}, b = {4, 3, 2, 1 - l};
  for (int it = 0; it < iters; ++it) {
    c0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, c3, 0, 0, 0);
  }
  long long s = 0;
  for (int r = 0; r < 16; ++r) s += (long long)c0[r] + c1[r] + c2[r] + c3[r];
  out[blockIdx.x * blockDim.x + l] = s;
}

}  // namespace

extern "C" int mpts_probe_rate(int32_t unit, double *per_second, void *out_dev, size_t out_bytes,
                               void *stream) {
  if (!per_second || !out_dev || (unit != MPTS_PROBE_VALU_MAD && unit != MPTS_PROBE_MFMA_I8))
    return MPTS_EINVAL;
  int dev = 0;
  hipDeviceProp_t pr;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess)
    return MPTS_EHIP;
  const int blocks = pr.multiProcessorCount * 4, threads = 256;
  if (out_bytes < (size_t)blocks * threads * 8) return MPTS_ENOSPC;
  hipStream_t s = (hipStream_t)stream;
  const int iters = unit == MPTS_PROBE_VALU_MAD ? 20000 : 4000;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MPTS_EHIP;
  float best = 0.f;
  for (int rep = 0; rep < 3; ++rep) {
    (void)hipEventRecord(e0, s);
    if (unit == MPTS_PROBE_VALU_MAD)
      hipLaunchKernelGGL(k_probe_mad, dim3(blocks), dim3(threads), 0, s, (long long *)out_dev, iters, rep);
    else
      hipLaunchKernelGGL(k_probe_mfma, dim3(blocks), dim3(threads), 0, s, (long long *)out_dev, iters, rep);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) return MPTS_EHIP;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (rep > 0 && (best == 0.f || ms < best)) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best <= 0.f) return MPTS_EHIP;
  const double ops = unit == MPTS_PROBE_VALU_MAD
                         ? (double)blocks * threads * iters * 64.0
                         : (double)blocks * (threads / 64) * iters * 4.0 * 32 * 32 * 32;
  *per_second = ops / (best * 1e-3);
  return MPTS_OK;
}
