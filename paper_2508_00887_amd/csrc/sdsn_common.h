// Reductions shared by the streaming and the on-chip SDSN kernels, so that
// both produce bit-identical partial sums, tile totals and maxima.
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

// Chain p of a row's and of a column's partial sums at once, for nb <= 16
// tiles, with the arithmetic of chain_sum.  All eight loads are issued before
// the first add (an index past the end is clamped to tile nb - 1 and its value
// dropped), so both chains together cost one memory round trip.
template <typename LoadR, typename LoadC>
__device__ __forceinline__ void chain_sum_pair16(LoadR ldr, LoadC ldc, int nb, int p, double& rs,
                                                 double& cs) {
  double rv[4], cv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = p + 4 * q;
    const int bc = b < nb ? b : nb - 1;
    rv[q] = ldr(bc);
    cv[q] = ldc(bc);
  }
  double ra = 0.0, ca = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const bool in = p + 4 * q < nb;
    ra = in ? ra + rv[q] : ra;
    ca = in ? ca + cv[q] : ca;
  }
  rs = ra;
  cs = ca;
}

__device__ __forceinline__ double combine4(double c0, double c1, double c2, double c3) {
  return (c0 + c1) + (c2 + c3);
}

// Global access at a uniform base plus a 32-bit element offset.  Written this
// way the address is an SGPR base plus a VGPR offset, so loop-invariant 64-bit
// per-lane addresses are never formed (and never spilled).
template <typename T>
__device__ __forceinline__ T& at_u32(T* base, unsigned off) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (size_t)(off * (unsigned)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const T& at_u32(const T* base, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                     (size_t)(off * (unsigned)sizeof(T)));
}

// Lane exchange inside a 16-lane DPP row, for one FP64 value.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// FP64 sum over the LPR lanes (16, 32 or 64) that hold one tile row, in a
// fixed order: a butterfly inside each 16-lane DPP row (neighbour, pair,
// half-row mirror, row mirror), then the DPP rows of the group in increasing
// order.  Every lane of the group receives the sum.  Must be reached by all
// 64 lanes of the wave (lanes outside the matrix pass 0).
template <int LPR>
__device__ __forceinline__ double row_group_sum(double v) {
  static_assert(LPR == 16 || LPR == 32 || LPR == 64, "row group of 16, 32 or 64 lanes");
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  if constexpr (LPR == 16) {
    return v;
  } else {
    const double r0 = readlane_f64(v, 0), r1 = readlane_f64(v, 16);
    const double r2 = readlane_f64(v, 32), r3 = readlane_f64(v, 48);
    if constexpr (LPR == 64) return (r0 + r1) + (r2 + r3);
    return (threadIdx.x & 32) ? r2 + r3 : r0 + r1;
  }
}

// Layout of a BM x BM tile over 4*BM threads: each wave holds 16 rows; a row
// is LPR = BM/4 lanes with four consecutive columns each; a wave step covers
// RPW = 64/LPR rows, so every thread visits STEPS = 16/RPW rows.
template <int BM>
struct TileShape {
  static constexpr int NT = 4 * BM;
  static constexpr int LPR = BM / 4;
  static constexpr int RPW = 64 / LPR;
  static constexpr int STEPS = 16 / RPW;
};

// Per-row contribution of one tile step: the row's FP64 sum (lane partials
// are FP32 sums of four entries) goes to s_rowsum[rl]; the column sums
// accumulate in cacc (FP32, at most 16 rows per lane).
template <int BM>
__device__ __forceinline__ void tile_step_sums(const float4& y, int rl, double* s_rowsum,
                                               float4& cacc) {
  const double rs = row_group_sum<TileShape<BM>::LPR>((double)((y.x + y.y) + (y.z + y.w)));
  if ((threadIdx.x & (TileShape<BM>::LPR - 1)) == 0) s_rowsum[rl] = rs;
  cacc.x += y.x;
  cacc.y += y.y;
  cacc.z += y.z;
  cacc.w += y.w;
}

// Plain stores (the streaming kernels: other workgroups read the values in a
// later launch).
struct PlainStore {
  template <typename T>
  __device__ __forceinline__ void operator()(T* p, T v) const { *p = v; }
};

// Writes the FP64 row partials, column partials and tile total of one tile
// from s_rowsum and the per-lane column sums cacc: rowp[bn * np + row],
// colp[bm * np + col], tot[bm * nb + bn].  s_colred holds 16 x BM floats.
// `st` performs the global stores.
template <int BM, typename Store = PlainStore>
__device__ __forceinline__ void tile_partials(const float4& cacc, const double* s_rowsum,
                                              float (*s_colred)[BM], double* s_red,
                                              double* rowp, double* colp, double* tot, int bm,
                                              int bn, int nb, int np, Store st = Store()) {
  using TS = TileShape<BM>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int q = lane / TS::LPR;
  const int cl = (lane % TS::LPR) * 4;
  *reinterpret_cast<float4*>(&s_colred[w * TS::RPW + q][cl]) = cacc;
  __syncthreads();
  double rowsum = 0.0;
  if (tid < BM) {
    rowsum = s_rowsum[tid];
    st(&at_u32(rowp, (unsigned)(bn * np + bm * BM + tid)), rowsum);
  }
  {  // column partials: 4 threads per column, fixed order, FP64
    const int c = tid >> 2, p = tid & 3;
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) v += (double)s_colred[p * 4 + u][c];
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    if (p == 0) st(&at_u32(colp, (unsigned)(bm * np + bn * BM + c)), v);
  }
  const double tt = block_sum<TS::NT>(rowsum, s_red);
  if (tid == 0) st(&tot[bm * nb + bn], tt);
}

}  // namespace
}  // namespace fram
