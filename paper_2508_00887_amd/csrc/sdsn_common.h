// Block reductions shared by the streaming and the on-chip SDSN kernels, so
// that both produce bit-identical tile totals and maxima.
#pragma once

#include <hip/hip_runtime.h>

namespace fram {
namespace {

// Block reductions: a butterfly inside each wave, then every thread adds the
// per-wave results in wave order.  The value is the same in every workgroup
// for the same inputs (fixed order), which the pass loop relies on.
template <int NT>
__device__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) r += sh[i];
  __syncthreads();
  return r;
}

template <int NT>
__device__ float block_max(float v, float* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = -INFINITY;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) r = fmaxf(r, sh[i]);
  __syncthreads();
  return r;
}

// Sum of base[b * stride] over the tiles b = p, p + 4, p + 8, ... < nb, in
// increasing b.  The full sum over b < nb is defined as
// (chain 0 + chain 1) + (chain 2 + chain 3); the streaming kernel forms the
// four chains in one thread, the on-chip kernel in four threads, with the
// same arithmetic.  Loads are issued four at a time before they are added.
template <typename LoadF>
__device__ __forceinline__ double chain_sum(LoadF load, int nb, int p) {
  double acc = 0.0;
  for (int b0 = p; b0 < nb; b0 += 16) {
    const double v0 = load(b0);
    const double v1 = (b0 + 4 < nb) ? load(b0 + 4) : 0.0;
    const double v2 = (b0 + 8 < nb) ? load(b0 + 8) : 0.0;
    const double v3 = (b0 + 12 < nb) ? load(b0 + 12) : 0.0;
    acc += v0;
    if (b0 + 4 < nb) acc += v1;
    if (b0 + 8 < nb) acc += v2;
    if (b0 + 12 < nb) acc += v3;
  }
  return acc;
}

__device__ __forceinline__ double combine4(double c0, double c1, double c2, double c3) {
  return (c0 + c1) + (c2 + c3);
}

}  // namespace
}  // namespace fram
