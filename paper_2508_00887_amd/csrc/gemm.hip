// MFMA GEMMs of the FRAM gradient X = A N B (Algorithm 1, step 5; eq. 3).
//
// Both products are written in "NT" form C = P * Q^T with P and Q row-major
// and K-contiguous: GEMM 1 is W = B * N^T (= (N B)^T because B is symmetric,
// Sec. 3) and GEMM 2 is X = A * W^T = A N B.  So every operand fragment is a
// contiguous 16-byte run of one row, loaded straight into LDS and read back
// with 128-bit LDS reads.
//
// Tiling for gfx950: a workgroup of 4 waves (2 x 2; 8 waves, 2 x 4, at
// BM = 256) owns a BM x BM output tile; each wave owns (BM/2) x (BM/2) (or
// 128 x 64) as a grid of 32 x 32 MFMA blocks
// (v_mfma_f32_32x32x16_{bf16,f16}, or four v_mfma_f32_32x32x2_f32 per 16-byte
// chunk for the FP32 path).  K advances 128 bytes of each row per step
// (64 bf16/f16 or 32 f32 elements) through a two-stage LDS ring with a
// register prefetch of the next stage.  LDS rows are 128 bytes; the 16-byte
// chunk index is XOR-swizzled with the row so the 128-bit reads of
// consecutive rows are free of bank conflicts.  Tiles are assigned so that the
// tiles of one XCD form a compact block of the tile grid (half its rows by a
// quarter of its columns), which keeps the row and column panels that XCD's
// L2 must hold few.
#include "fram_internal.h"

namespace fram {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
// 16-byte fragment as a native vector: arrays of these are kept in VGPRs.
typedef unsigned v4u __attribute__((ext_vector_type(4)));

template <Elem E>
struct Mfma;

template <>
struct Mfma<Elem::BF16> {
  static constexpr int kPerChunk = 8;
  __device__ static inline void mac(const v4u& a, const v4u& b, f32x16& c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
  __device__ static inline void store(void* C, size_t idx, float v) {
    reinterpret_cast<__bf16*>(C)[idx] = static_cast<__bf16>(v);
  }
};

template <>
struct Mfma<Elem::F16> {
  static constexpr int kPerChunk = 8;
  __device__ static inline void mac(const v4u& a, const v4u& b, f32x16& c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  }
  __device__ static inline void store(void* C, size_t idx, float v) {
    reinterpret_cast<_Float16*>(C)[idx] = static_cast<_Float16>(v);
  }
};

template <>
struct Mfma<Elem::F32> {
  static constexpr int kPerChunk = 4;
  // Lane l holds A[row l%32][k-slot l/32] per instruction; the four floats of
  // the chunk are four k-slots, applied identically to the A and B fragments.
  __device__ static inline void mac(const v4u& a, const v4u& b, f32x16& c) {
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
  }
  __device__ static inline void store(void* C, size_t idx, float v) {
    reinterpret_cast<float*>(C)[idx] = v;
  }
};

constexpr int kChunks = 8;  // 16-byte chunks per LDS row (128 bytes of K)

// LDS has 64 four-byte banks: 16 lanes of a 128-bit read cover all of them
// when the 16 consecutive rows they read (two rows per 256 bytes) put their
// chunk in 8 different places per row parity.
__device__ __forceinline__ int swz(int row, int ch) { return ch ^ ((row >> 1) & 7); }

// Waves per workgroup: a 2 x (NW / 2) grid of waves over the output tile.
// At BM = 256 eight waves (128 x 64 each, 128 accumulator registers) put two
// waves on every SIMD, so one wave's MFMAs run while the other waits for
// memory; four waves of 128 x 128 would leave each SIMD idle for the whole of
// every read that misses the L2.
template <int BM>
constexpr int gemm_waves() {
  return BM == 256 ? 8 : 4;
}

// Output tile (tm, tn) of C = P * Q^T: one workgroup of 64 * gemm_waves<BM>
// threads.
template <Elem E, int BM, bool OUT_F32>
__device__ __forceinline__ void gemm_tile(const v4u* __restrict__ P, const v4u* __restrict__ Q,
                                          void* __restrict__ C, const float* __restrict__ bias,
                                          int ld, int ktiles, int tm, int tn) {
  constexpr int NW = gemm_waves<BM>();
  constexpr int NT = 64 * NW;
  constexpr int WTM = BM / 2;          // wave tile rows
  constexpr int WTN = BM / (NW / 2);   // wave tile columns
  constexpr int FM = WTM / 32;         // MFMA blocks per wave tile, rows
  constexpr int FN = WTN / 32;         // ... and columns
  constexpr int RPL = NT / kChunks;    // rows one load step covers
  constexpr int LOADS = BM / RPL;
  __shared__ v4u smem[2][2][BM][kChunks];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m0 = tm * BM;
  const int n0 = tn * BM;
  const int wm = wave / (NW / 2), wn = wave % (NW / 2);
  const int ldc = ld / Mfma<E>::kPerChunk;  // leading dimension in chunks

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

  const int lrow = tid / kChunks;  // 0 .. RPL - 1
  const int lch = tid % kChunks;
  const int half = lane >> 5;
  const int l32 = lane & 31;
  const v4u* pg = P + (size_t)(m0 + lrow) * ldc + lch;
  const v4u* qg = Q + (size_t)(n0 + lrow) * ldc + lch;
  const size_t rstep = (size_t)RPL * ldc;  // RPL rows further down

  // Prefetch registers for the next K tile.  No lambdas here: an array that a
  // lambda captures by reference is kept in scratch memory.
  v4u ra[LOADS], rb[LOADS];
#pragma unroll
  for (int i = 0; i < LOADS; ++i) {
    ra[i] = pg[i * rstep];
    rb[i] = qg[i * rstep];
  }
#pragma unroll
  for (int i = 0; i < LOADS; ++i) {
    const int r = lrow + RPL * i;
    smem[0][0][r][swz(r, lch)] = ra[i];
    smem[0][1][r][swz(r, lch)] = rb[i];
  }
  __syncthreads();

  for (int kt = 0; kt < ktiles; ++kt) {
    const int st = kt & 1;
    const bool more = kt + 1 < ktiles;
    if (more) {
      const size_t ko = (size_t)(kt + 1) * kChunks;
#pragma unroll
      for (int i = 0; i < LOADS; ++i) {
        ra[i] = pg[i * rstep + ko];
        rb[i] = qg[i * rstep + ko];
      }
    }
    // Fragments of step s + 1 are read from LDS while step s runs on MFMA.
    v4u a[2][FM], b[2][FN];
#pragma unroll
    for (int f = 0; f < FM; ++f) {
      const int ra_ = wm * WTM + f * 32 + l32;
      a[0][f] = smem[st][0][ra_][swz(ra_, half)];
    }
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int rb_ = wn * WTN + f * 32 + l32;
      b[0][f] = smem[st][1][rb_][swz(rb_, half)];
    }
#pragma unroll
    for (int s = 0; s < kChunks / 2; ++s) {
      const int cur = s & 1;
      if (s + 1 < kChunks / 2) {
        const int ch = 2 * (s + 1) + half;
#pragma unroll
        for (int f = 0; f < FM; ++f) {
          const int ra_ = wm * WTM + f * 32 + l32;
          a[cur ^ 1][f] = smem[st][0][ra_][swz(ra_, ch)];
        }
#pragma unroll
        for (int f = 0; f < FN; ++f) {
          const int rb_ = wn * WTN + f * 32 + l32;
          b[cur ^ 1][f] = smem[st][1][rb_][swz(rb_, ch)];
        }
      }
      // Keep those reads ahead of this step's MFMAs (the scheduler would
      // otherwise sink each read next to its first use and expose the LDS
      // latency); for FP32 its own order measured slightly faster.
      if constexpr (E != Elem::F32) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) Mfma<E>::mac(a[cur][i], b[cur][j], acc[i][j]);
      if constexpr (E != Elem::F32) __builtin_amdgcn_sched_barrier(0);
    }
    if (more) {
#pragma unroll
      for (int i = 0; i < LOADS; ++i) {
        const int r = lrow + RPL * i;
        smem[st ^ 1][0][r][swz(r, lch)] = ra[i];
        smem[st ^ 1][1][r][swz(r, lch)] = rb[i];
      }
    }
    __syncthreads();
  }

  // Accumulator layout of a 32x32 MFMA block: element 4*g + r of lane l is
  // row 8*g + 4*(l/32) + r, column l%32.
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const size_t row = (size_t)(m0 + wm * WTM + i * 32 + 8 * g + 4 * half + r);
          const size_t col = (size_t)(n0 + wn * WTN + j * 32 + l32);
          float v = acc[i][j][4 * g + r];
          if (OUT_F32 && bias != nullptr) v += bias[row * ld + col];
          if (OUT_F32)
            reinterpret_cast<float*>(C)[row * ld + col] = v;
          else
            Mfma<E>::store(C, row * ld + col, v);
        }
}

template <Elem E, int BM, bool OUT_F32>
__global__ __launch_bounds__(64 * gemm_waves<BM>()) void gemm_nt_kernel(
    const v4u* __restrict__ P, const v4u* __restrict__ Q, void* __restrict__ C,
    const float* __restrict__ bias, int np, int ld, int ktiles) {
  const int nbn = np / BM;
  const int bid = blockIdx.x;
  const int ntiles = gridDim.x;
  int tm = bid / nbn, tn = bid % nbn;
  if ((ntiles & 7) == 0 && (nbn & 1) == 0 && ((nbn / 2) & 3) == 0) {
    // Workgroup bid runs on XCD bid % 8.  XCD x takes the x-th block of the
    // tile grid cut into 2 x 4 blocks (nbn/2 tile rows by nbn/4 tile columns).
    const int x = bid & 7, k = bid >> 3;
    const int bh = nbn / 2, bw = nbn / 4;
    tm = (x >> 2) * bh + k / bw;
    tn = (x & 3) * bw + k % bw;
  }
  gemm_tile<E, BM, OUT_F32>(P, Q, C, bias, ld, ktiles, tm, tn);
}

// Many independent products (one job each, blockIdx.y), each one tile of
// edge BM (np == BM): the GEMMs of a group of small pairs in one launch.
template <Elem E, int BM, bool OUT_F32>
__global__ __launch_bounds__(64 * gemm_waves<BM>()) void gemm_group_kernel(
    const GemmJob* __restrict__ jobs) {
  const GemmJob j = jobs[blockIdx.y];
  gemm_tile<E, BM, OUT_F32>(static_cast<const v4u*>(j.P), static_cast<const v4u*>(j.Q), j.C,
                            nullptr, j.ld, j.ktiles, 0, 0);
}

template <Elem E, bool OUT_F32>
hipError_t launch_group_e(int bm, const GemmJob* jobs, int count, hipStream_t s) {
  const dim3 grid(1, count);
  switch (bm) {
    case 64:
      gemm_group_kernel<E, 64, OUT_F32><<<grid, 64 * gemm_waves<64>(), 0, s>>>(jobs);
      break;
    case 128:
      gemm_group_kernel<E, 128, OUT_F32><<<grid, 64 * gemm_waves<128>(), 0, s>>>(jobs);
      break;
    case 256:
      gemm_group_kernel<E, 256, OUT_F32><<<grid, 64 * gemm_waves<256>(), 0, s>>>(jobs);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <Elem E, bool OUT_F32>
hipError_t launch_e(int bm, const void* P, const void* Q, void* C, const float* bias, int n,
                    int np, int ld, hipStream_t s) {
  const int kelems = kChunks * Mfma<E>::kPerChunk;
  const int ktiles = (n + kelems - 1) / kelems;
  const int nb = np / bm;
  dim3 grid(nb * nb);
  const v4u* p = static_cast<const v4u*>(P);
  const v4u* q = static_cast<const v4u*>(Q);
  switch (bm) {
    case 64:
      gemm_nt_kernel<E, 64, OUT_F32><<<grid, 64 * gemm_waves<64>(), 0, s>>>(p, q, C, bias, np, ld,
                                                                           ktiles);
      break;
    case 128:
      gemm_nt_kernel<E, 128, OUT_F32><<<grid, 64 * gemm_waves<128>(), 0, s>>>(p, q, C, bias, np,
                                                                             ld, ktiles);
      break;
    case 256:
      gemm_nt_kernel<E, 256, OUT_F32><<<grid, 64 * gemm_waves<256>(), 0, s>>>(p, q, C, bias, np,
                                                                             ld, ktiles);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

int gemm_ktiles(Elem e, int n) {
  const int kelems = kChunks * (e == Elem::F32 ? 4 : 8);
  return (n + kelems - 1) / kelems;
}

hipError_t launch_gemm_group(Elem e, int bm, bool c_f32, const GemmJob* jobs, int count,
                             hipStream_t s) {
  if (count < 1) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  switch (e) {
    case Elem::F32:  // FP32 products are always written as float
      return launch_group_e<Elem::F32, true>(bm, jobs, count, s);
    case Elem::BF16:
      return c_f32 ? launch_group_e<Elem::BF16, true>(bm, jobs, count, s)
                   : launch_group_e<Elem::BF16, false>(bm, jobs, count, s);
    case Elem::F16:
      return c_f32 ? launch_group_e<Elem::F16, true>(bm, jobs, count, s)
                   : launch_group_e<Elem::F16, false>(bm, jobs, count, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_nt(Elem e, int bm, const void* P, const void* Q, void* C, bool c_f32,
                          int n, int np, int ld, hipStream_t s, const float* bias) {
  if (np % bm != 0 || ld < np || np % 64 != 0 || n > np) return hipErrorInvalidValue;
  if (bias != nullptr && !c_f32) return hipErrorInvalidValue;
  switch (e) {
    case Elem::F32:
      return launch_e<Elem::F32, true>(bm, P, Q, C, bias, n, np, ld, s);
    case Elem::BF16:
      return c_f32 ? launch_e<Elem::BF16, true>(bm, P, Q, C, bias, n, np, ld, s)
                   : launch_e<Elem::BF16, false>(bm, P, Q, C, bias, n, np, ld, s);
    case Elem::F16:
      return c_f32 ? launch_e<Elem::F16, true>(bm, P, Q, C, bias, n, np, ld, s)
                   : launch_e<Elem::F16, false>(bm, P, Q, C, bias, n, np, ld, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace fram
