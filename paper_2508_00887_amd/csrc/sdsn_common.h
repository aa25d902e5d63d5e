// Reductions shared by the streaming and the on-chip SDSN kernels, so that
// both produce bit-identical partial sums, tile totals and maxima.
#pragma once

#include <hip/hip_runtime.h>

namespace fram {
namespace {

// ---- Cross-lane moves (64-lane waves).

// DPP move inside 16-lane rows, for one FP64 value; every source lane of the
// controls used here is valid.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
constexpr int kDppXor1 = 0xB1;      // quad_perm [1,0,3,2]: lane ^ 1
constexpr int kDppXor2 = 0x4E;      // quad_perm [2,3,0,1]: lane ^ 2
constexpr int kDppXor8 = 0x128;     // row_ror:8 inside a 16-lane row: lane ^ 8
constexpr int kDppHalfMirror = 0x141;  // lane 8k+i <-> lane 8k+7-i (pairs bit-2 halves)

// Exchange between two registers by lane blocks (gfx950 permlane swaps).
// swap32: a = [a_lo | b_lo], b = [a_hi | b_hi] by 32-lane halves.
// swap16: a = [a0 b0 a2 b2], b = [a1 b1 a3 b3] by 16-lane rows.
__device__ __forceinline__ void swap32_f64(double& a, double& b) {
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi =
      __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  const unsigned long long na = ((unsigned long long)hi[0] << 32) | lo[0];
  const unsigned long long nb = ((unsigned long long)hi[1] << 32) | lo[1];
  a = __builtin_bit_cast(double, na);
  b = __builtin_bit_cast(double, nb);
}
__device__ __forceinline__ void swap16_f64(double& a, double& b) {
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi =
      __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  const unsigned long long na = ((unsigned long long)hi[0] << 32) | lo[0];
  const unsigned long long nb = ((unsigned long long)hi[1] << 32) | lo[1];
  a = __builtin_bit_cast(double, na);
  b = __builtin_bit_cast(double, nb);
}
// (The vector elements are copied to scalars before the bit casts: this
// compiler's __builtin_bit_cast of an element of an ext_vector_type reads
// element 0 whatever the index.)
__device__ __forceinline__ void swap32_f32(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a),
                                                  __builtin_bit_cast(unsigned, b), false, false);
  const unsigned r0 = r[0], r1 = r[1];
  a = __builtin_bit_cast(float, r0);
  b = __builtin_bit_cast(float, r1);
}
__device__ __forceinline__ void swap16_f32(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a),
                                                  __builtin_bit_cast(unsigned, b), false, false);
  const unsigned r0 = r[0], r1 = r[1];
  a = __builtin_bit_cast(float, r0);
  b = __builtin_bit_cast(float, r1);
}

// One step of a transposing pairwise sum at lane bit B (5 ... 2): the lanes
// whose bit B is 0 return a + (a of their partner lane), the others
// b + (b of theirs); the partner differs in bit B only (in the half-row
// mirror's pairing for B = 2).  Two values per lane become one, and no lane's
// work is wasted.
template <int B>
__device__ __forceinline__ double pair_step(double a, double b) {
  static_assert(B >= 2 && B <= 5, "lane bits 2-5");
  if constexpr (B == 5) {
    swap32_f64(a, b);
    return a + b;
  } else if constexpr (B == 4) {
    swap16_f64(a, b);
    return a + b;
  } else {
    const bool up = (threadIdx.x >> B) & 1;
    const double send = up ? a : b;
    const double keep = up ? b : a;
    return keep + dpp_f64<B == 3 ? kDppXor8 : kDppHalfMirror>(send);
  }
}

// Sum (max) over the 64 lanes of a wave in a fixed pairing order (bit 5, 4,
// 3, the half-row mirror, bits 1 and 0); every lane receives the result.
__device__ __forceinline__ double wave_sum_f64(double v) {
  double t = v;
  swap32_f64(v, t);
  v = v + t;
  t = v;
  swap16_f64(v, t);
  v = v + t;
  v += dpp_f64<kDppXor8>(v);
  v += dpp_f64<kDppHalfMirror>(v);
  v += dpp_f64<kDppXor2>(v);
  v += dpp_f64<kDppXor1>(v);
  return v;
}
__device__ __forceinline__ float wave_max_f32(float v) {
  float t = v;
  swap32_f32(v, t);
  v = fmaxf(v, t);
  t = v;
  swap16_f32(v, t);
  v = fmaxf(v, t);
  v = fmaxf(v, dpp_f32<kDppXor8>(v));
  v = fmaxf(v, dpp_f32<kDppHalfMirror>(v));
  v = fmaxf(v, dpp_f32<kDppXor2>(v));
  v = fmaxf(v, dpp_f32<kDppXor1>(v));
  return v;
}

// Block reductions: the wave sums above, then every thread adds the per-wave
// results in wave order.  The value is the same in every workgroup for the
// same inputs (fixed order), which the pass loop relies on.
template <int NT>
__device__ double block_sum(double v, double* sh) {
  v = wave_sum_f64(v);
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
  v = wave_max_f32(v);
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
// A wave-uniform double held in scalar registers (its two halves read from
// the first lane).
__device__ __forceinline__ double uniform_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readfirstlane((int)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

template <typename T>
__device__ __forceinline__ T& at_u32(T* base, unsigned off) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (size_t)(off * (unsigned)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ const T& at_u32(const T* base, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) +
                                     (size_t)(off * (unsigned)sizeof(T)));
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

// FP64 row sums of a wave's 16 tile rows, formed all at once.  Step stp of a
// lane contributes the FP32 sum of its four entries of row
// w*16 + stp*RPW + lane/LPR.  The sums over the LPR lanes of each row are
// built as a pairwise tree whose level l joins steps differing in bit l at
// lane bit TOP - l (pair_step): the two values of a lane become one, so the
// STEPS values per lane shrink to one, level by level, as the steps arrive
// (at most LEVELS values wait at any time).  The lane then holds step
// s = sum_l bit(lane, TOP - l) << l of its row group, summed over the lanes
// that differ in bits TOP ... 2; bits 1 and 0 are added last, so all four
// lanes of a quad hold the row's sum.
template <int BM>
struct RowSums {
  using TS = TileShape<BM>;
  static constexpr int LEVELS = TS::STEPS == 16 ? 4 : (TS::STEPS == 8 ? 3 : 2);
  static constexpr int TOP = LEVELS + 1;  // lane bit of level 0: 5, 4 or 3
  static_assert((1 << LEVELS) == TS::STEPS && (2 << TOP) == TS::LPR, "tile shape");
  double pend[LEVELS];
  double sum;

  // Step stp (a compile-time constant once the step loop is unrolled).
  __device__ __forceinline__ void push(int stp, const float4& y) {
    carry<0>(stp, (double)((y.x + y.y) + (y.z + y.w)));
  }
  template <int L>
  __device__ __forceinline__ void carry(int stp, double v) {
    if constexpr (L == LEVELS) {
      sum = v;
    } else {
      if (((stp >> L) & 1) == 0) {
        pend[L] = v;
        return;
      }
      carry<L + 1>(stp, pair_step<TOP - L>(pend[L], v));
    }
  }
  // After the last step: s_rowsum[row] for the wave's 16 rows.
  __device__ __forceinline__ void finish(int w, double* s_rowsum) const {
    double v = sum;
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    const int lane = threadIdx.x & 63;
    int s = 0;
#pragma unroll
    for (int l = 0; l < LEVELS; ++l) s |= ((lane >> (TOP - l)) & 1) << l;
    if ((lane & 3) == 0) s_rowsum[w * 16 + s * TS::RPW + lane / TS::LPR] = v;
  }
};

// One tile step's contribution to the sums: its row partials (RowSums) and
// the lane's column sums cacc (FP32, at most 16 rows per lane).
template <int BM>
__device__ __forceinline__ void tile_step_sums(const float4& y, int stp, RowSums<BM>& rows,
                                               float4& cacc) {
  rows.push(stp, y);
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
                                              int bn, int nb, int np, Store st = Store(),
                                              int tid = (int)threadIdx.x) {
  using TS = TileShape<BM>;
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
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    if (p == 0) st(&at_u32(colp, (unsigned)(bm * np + bn * BM + c)), v);
  }
  const double tt = block_sum<TS::NT>(rowsum, s_red);
  if (tid == 0) st(&at_u32(tot, (unsigned)(bm * nb + bn)), tt);
}

}  // namespace
}  // namespace fram
