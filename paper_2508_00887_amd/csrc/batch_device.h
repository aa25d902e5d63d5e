// Batched FRAM: many independent graph pairs of uneven size in one persistent
// launch (Algorithm 1 with Algorithm 2 per pair).
//
// Each workgroup (256 lanes) pulls the next pair from a queue ordered by
// decreasing n and runs the whole solve for it: prescale (Alg. 1 steps 2-3),
// the outer loop (step 5 GEMMs on MFMA, step 6 SDSN passes, steps 7-8 update
// and delta), the row argmax with a permutation check (step 10; when rows
// collide, the exact assignment of lap_device.h in the workgroup's LDS) and
// the FP64 objective.  A pair never needs more than one workgroup (n <= 512), so every
// reduction is workgroup-local, fixed-order and free of grid barriers, and a
// pair's result does not depend on which workgroup ran it or on the other
// pairs in the batch.
//
// Matrices live in one arena (np x np, np = n rounded up to 32, zero padded).
// The GEMMs read their operands straight from L2 in 16-byte fragments; each
// wave owns 32 x 32 output tiles.  An SDSN pass streams X once: waves take
// 16-row blocks, lanes take float4 column chunks; row sums go through an LDS
// transpose, column sums accumulate per lane and are combined across waves in
// FP64.  The pass arithmetic is the one of the single-pair kernels:
// Y = max(0, fma(s, x, alpha_i + beta_j)) with the symmetric FP64 split of
// the P1 correction (eq. P1_sol), gamma in FP64 (Sec. 5.2).
#pragma once

#include "fram_internal.h"
#include "lap_device.h"

namespace fram {
namespace {

constexpr int kBT = 256;
constexpr int kW = kBT / 64;  // waves per workgroup
constexpr int kRB = 16;       // rows per wave block in a pass

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <Elem E>
struct BT;
template <>
struct BT<Elem::BF16> {
  typedef __bf16 T;
  static constexpr int kStep = 16;
  __device__ static void mac(const uint4& a, const uint4& b, f32x16& c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
  __device__ static T cvt(float v) { return (__bf16)v; }
};
template <>
struct BT<Elem::F16> {
  typedef _Float16 T;
  static constexpr int kStep = 16;
  __device__ static void mac(const uint4& a, const uint4& b, f32x16& c) {
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a),
                                                __builtin_bit_cast(f16x8, b), c, 0, 0, 0);
  }
  __device__ static T cvt(float v) { return (_Float16)v; }
};
template <>
struct BT<Elem::F32> {
  typedef float T;
  static constexpr int kStep = 8;
  __device__ static void mac(const uint4& a, const uint4& b, f32x16& c) {
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
  }
  __device__ static T cvt(float v) { return v; }
};

struct Shared {
  double r[kBatchMaxN];         // row sums of the current iterate
  double c[kBatchMaxN];         // column sums of the current iterate
  float a[kBatchMaxN];          // alpha_i
  float b[kBatchMaxN];          // beta_j
  float tr[kW][kRB][65];        // row-partial transpose, one block per wave
  double cp[kW][kBatchMaxN];    // per-wave column partials
  double red[kW];
  float redf[kW];
  int hits[kBatchMaxN];
  int flag;
  int same;
};

__device__ double wg_sum(double v, Shared& sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < kW; ++i) r += sh.red[i];
  __syncthreads();
  return r;
}

__device__ float wg_max(float v, Shared& sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) sh.redf[threadIdx.x >> 6] = v;
  __syncthreads();
  float r = -INFINITY;
#pragma unroll
  for (int i = 0; i < kW; ++i) r = fmaxf(r, sh.redf[i]);
  __syncthreads();
  return r;
}

// C (np x np) = P Q^T on MFMA; OUT_F32 stores float, else the GEMM type.
template <Elem E, bool OUT_F32>
__device__ void wg_gemm_nt(const typename BT<E>::T* __restrict__ P,
                           const typename BT<E>::T* __restrict__ Q, void* __restrict__ C,
                           int np) {
  typedef typename BT<E>::T T;
  constexpr int S = BT<E>::kStep;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int l32 = lane & 31, half = lane >> 5;
  const int tn = np / 32, tiles = tn * tn;
  for (int t = w; t < tiles; t += kW) {
    const int tm = t / tn, tc = t % tn;
    const T* pr = P + (size_t)(tm * 32 + l32) * np + half * (S / 2);
    const T* qr = Q + (size_t)(tc * 32 + l32) * np + half * (S / 2);
    f32x16 acc;
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
#pragma unroll 4
    for (int k = 0; k < np; k += S) {
      const uint4 av = *reinterpret_cast<const uint4*>(pr + k);
      const uint4 bv = *reinterpret_cast<const uint4*>(qr + k);
      BT<E>::mac(av, bv, acc);
    }
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t row = (size_t)(tm * 32 + 8 * g + 4 * half + r);
        const size_t idx = row * np + tc * 32 + l32;
        if (OUT_F32)
          reinterpret_cast<float*>(C)[idx] = acc[4 * g + r];
        else
          reinterpret_cast<T*>(C)[idx] = BT<E>::cvt(acc[4 * g + r]);
      }
  }
}

// One sweep over X (rows < n): PASS = false collects row/column sums and the
// max of X; PASS = true applies one SDSN pass with scale s in place and
// collects the sums of the result.  Sums land in sh.r / sh.c; returns the
// FP64 total (and the max through *mx for the statistics sweep).
template <bool PASS>
__device__ double wg_sweep(float* __restrict__ X, int n, int np, float s, Shared& sh,
                           float* mx) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nch = np / 4;
  const int c0 = lane, c1 = lane + 64;
  const bool h0 = c0 < nch, h1 = c1 < nch;
  double cacc0[4] = {0, 0, 0, 0}, cacc1[4] = {0, 0, 0, 0};
  float lmax = -INFINITY;
  for (int rb0 = 0; rb0 < n; rb0 += kW * kRB) {
    float cb0[4] = {0, 0, 0, 0}, cb1[4] = {0, 0, 0, 0};
    for (int rr = 0; rr < kRB; ++rr) {
      const int i = rb0 + w * kRB + rr;
      float rowp = 0.0f;
      if (i < n) {
        const float ai = PASS ? sh.a[i] : 0.0f;
#pragma unroll
        for (int hsel = 0; hsel < 2; ++hsel) {
          const int ch = hsel ? c1 : c0;
          if (!(hsel ? h1 : h0)) continue;
          const int j = 4 * ch;
          float4* p = reinterpret_cast<float4*>(X + (size_t)i * np + j);
          float4 y = *p;
          if (PASS) {
            y.x = (j < n) ? fmaxf(0.0f, fmaf(s, y.x, ai + sh.b[j])) : 0.0f;
            y.y = (j + 1 < n) ? fmaxf(0.0f, fmaf(s, y.y, ai + sh.b[j + 1])) : 0.0f;
            y.z = (j + 2 < n) ? fmaxf(0.0f, fmaf(s, y.z, ai + sh.b[j + 2])) : 0.0f;
            y.w = (j + 3 < n) ? fmaxf(0.0f, fmaf(s, y.w, ai + sh.b[j + 3])) : 0.0f;
            *p = y;
          } else {
            y.x = (j < n) ? y.x : 0.0f;
            y.y = (j + 1 < n) ? y.y : 0.0f;
            y.z = (j + 2 < n) ? y.z : 0.0f;
            y.w = (j + 3 < n) ? y.w : 0.0f;
            if (j < n) lmax = fmaxf(lmax, y.x);
            if (j + 1 < n) lmax = fmaxf(lmax, y.y);
            if (j + 2 < n) lmax = fmaxf(lmax, y.z);
            if (j + 3 < n) lmax = fmaxf(lmax, y.w);
          }
          rowp += (y.x + y.y) + (y.z + y.w);
          float* cb = hsel ? cb1 : cb0;
          cb[0] += y.x;
          cb[1] += y.y;
          cb[2] += y.z;
          cb[3] += y.w;
        }
      }
      sh.tr[w][rr][lane] = rowp;
    }
    __syncthreads();
    {  // row sums of this block: 4 lanes per row, FP64, fixed order
      const int rr = lane >> 2, part = lane & 3;
      double v = 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) v += (double)sh.tr[w][rr][part * 16 + u];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      const int i = rb0 + w * kRB + rr;
      if (part == 0 && i < n) sh.r[i] = v;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      cacc0[e] += (double)cb0[e];
      cacc1[e] += (double)cb1[e];
    }
    __syncthreads();
  }
  // Column sums: per-wave partials, then a fixed-order combine.
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (h0) sh.cp[w][4 * c0 + e] = cacc0[e];
    if (h1) sh.cp[w][4 * c1 + e] = cacc1[e];
  }
  __syncthreads();
  for (int j = tid; j < np; j += kBT) {
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < kW; ++q) v += sh.cp[q][j];
    sh.c[j] = (j < n) ? v : 0.0;
  }
  double part = 0.0;
  for (int i = tid; i < n; i += kBT) part += sh.r[i];
  const double S = wg_sum(part, sh);  // synchronises: sh.c and sh.r are complete
  if (!PASS) *mx = wg_max(lmax, sh);
  return S;
}

// Row argmax of N (lowest column on ties) into sigma; sh.flag = 1 if it is a
// permutation.  With prev != nullptr also compares with prev (returns 1 if
// equal) and then copies sigma into prev.
__device__ int wg_argmax(const float* __restrict__ Nf, int n, int np, int32_t* __restrict__ sigma,
                         int32_t* __restrict__ prev, Shared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int j = tid; j < n; j += kBT) sh.hits[j] = 0;
  if (tid == 0) sh.same = 1;
  __syncthreads();
  for (int i = w; i < n; i += kW) {
    const float* row = Nf + (size_t)i * np;
    float best = -INFINITY;
    int bi = n;
    for (int j = lane; j < n; j += 64) {
      const float v = row[j];
      if (v > best) {
        best = v;
        bi = j;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const float ob = __shfl_xor(best, o);
      const int oi = __shfl_xor(bi, o);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      const int j = bi < n ? bi : 0;
      sigma[i] = j;
      atomicAdd(&sh.hits[j], 1);
      if (prev != nullptr) {
        if (prev[i] != j) sh.same = 0;
        prev[i] = j;
      }
    }
  }
  __syncthreads();
  if (tid == 0) sh.flag = 1;
  __syncthreads();
  for (int j = tid; j < n; j += kBT)
    if (sh.hits[j] != 1) sh.flag = 0;
  __syncthreads();
  const int same = sh.same;
  __syncthreads();
  return same;
}

template <Elem E>
__device__ void solve_pair(const BatchArgs& A, const BatchPair& P, BatchResult& R, Shared& sh,
                           LapShared<kW>& lsh) {
  typedef typename BT<E>::T T;
  const int n = P.n, np = P.np, tid = threadIdx.x;
  const double* A64 = reinterpret_cast<const double*>(A.arena + P.a64);
  const double* B64 = reinterpret_cast<const double*>(A.arena + P.b64);
  T* Alp = reinterpret_cast<T*>(A.arena + P.alp);
  T* Blp = reinterpret_cast<T*>(A.arena + P.blp);
  T* W = reinterpret_cast<T*>(A.arena + P.w);
  float* Nf = reinterpret_cast<float*>(A.arena + P.nf);
  T* Nlp = (E == Elem::F32) ? reinterpret_cast<T*>(Nf) : reinterpret_cast<T*>(A.arena + P.nlp);
  float* X = reinterpret_cast<float*>(A.arena + P.x);
  int32_t* sigma = reinterpret_cast<int32_t*>(A.arena + P.sigma);
  const size_t nn = (size_t)n * n, npp = (size_t)np * np;

  {
    // Algorithm 1 steps 2-3: each matrix scaled by its own maximum.
    double ma = -INFINITY, mb = -INFINITY;
    for (size_t t = tid; t < nn; t += kBT) {
      ma = fmax(ma, A64[t]);
      mb = fmax(mb, B64[t]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      ma = fmax(ma, __shfl_xor(ma, o));
      mb = fmax(mb, __shfl_xor(mb, o));
    }
    if ((tid & 63) == 0) {
      sh.red[tid >> 6] = ma;
      sh.cp[0][tid >> 6] = mb;
    }
    __syncthreads();
    ma = -INFINITY;
    mb = -INFINITY;
    for (int q = 0; q < kW; ++q) {
      ma = fmax(ma, sh.red[q]);
      mb = fmax(mb, sh.cp[0][q]);
    }
    __syncthreads();
    const double da = ma > 0.0 ? ma : 1.0, db = mb > 0.0 ? mb : 1.0;
    const double ka = ma > 0.0 ? 1.0 : 0.0, kb = mb > 0.0 ? 1.0 : 0.0;
    for (size_t t = tid; t < npp; t += kBT) {
      const int i = (int)(t / np), j = (int)(t % np);
      const bool in = i < n && j < n;
      Alp[t] = BT<E>::cvt(in ? (float)(ka * (A64[(size_t)i * n + j] / da)) : 0.0f);
      Blp[t] = BT<E>::cvt(in ? (float)(kb * (B64[(size_t)i * n + j] / db)) : 0.0f);
      Nf[t] = 0.0f;
      if (E != Elem::F32) Nlp[t] = BT<E>::cvt(0.0f);
    }
    __syncthreads();

    const double dn = (double)n;
    const float alpha = (float)A.alpha, c1a = 1.0f - (float)A.alpha;
    int it = 0, total = 0, pmax = 0, plast = 0, capped = 0, converged = 0;
    int stable = 0;
    bool prev_perm = false, tracked = false;
    int32_t* sigprev = reinterpret_cast<int32_t*>(A.arena + P.sigprev);
    double delta = 0.0, gamma = 0.0;
    for (it = 1; it <= A.iters; ++it) {
      // Step 5: W = B N^T, X = A W^T.
      wg_gemm_nt<E, false>(Blp, Nlp, W, np);
      __syncthreads();
      wg_gemm_nt<E, true>(Alp, W, X, np);
      __syncthreads();
      // Step 6: SDSN (Algorithm 2) in place on X.
      float mx = 0.0f;
      double S = wg_sweep<false>(X, n, np, 1.0f, sh, &mx);
      float s = (mx > 0.0f) ? (float)(A.theta / (2.0 * (double)mx)) : 0.0f;
      int k = 0;
      while (true) {
        const double sd = (double)s;
        const double hf = 0.5 / dn + 0.5 * sd * S / (dn * dn);
        for (int j = tid; j < np; j += kBT) {
          sh.a[j] = (float)(hf - sd * sh.r[j] / dn);
          sh.b[j] = (float)(hf - sd * sh.c[j] / dn);
        }
        __syncthreads();
        S = wg_sweep<true>(X, n, np, s, sh, nullptr);
        ++k;
        s = 1.0f;
        gamma = S / dn - 1.0;
        if (gamma <= A.gamma_tol || k >= A.sdsn_max) break;
      }
      total += k;
      plast = k;
      pmax = k > pmax ? k : pmax;
      if (k >= A.sdsn_max && !(gamma <= A.gamma_tol)) capped = 1;
      // Steps 7-8: N <- (1-alpha) N + alpha D, delta in FP64.
      double num = 0.0, den = 0.0;
      for (size_t t = tid; t < (size_t)n * np; t += kBT) {
        const float o = Nf[t], d = X[t];
        const float v = fmaf(alpha, d, c1a * o);
        Nf[t] = v;
        if (E != Elem::F32) Nlp[t] = BT<E>::cvt(v);
        const double e = (double)v - (double)o;
        num += e * e;
        den += (double)v * v;
      }
      num = wg_sum(num, sh);
      den = wg_sum(den, sh);
      delta = den > 0.0 ? sqrt(num) / sqrt(den) : 0.0;
      tracked = false;
      if (delta <= A.tol) {
        converged = 1;
        break;
      }
      if (!isfinite(delta) || !isfinite(gamma)) break;
      if (A.stable_iters > 0) {
        // Argmax-stability stop (same rule as the single-pair path).
        const int same = wg_argmax(Nf, n, np, sigma, sigprev, sh);
        tracked = true;
        const bool is_perm = sh.flag != 0;
        stable = (is_perm && prev_perm && same) ? stable + 1 : 0;
        prev_perm = is_perm;
        if (stable >= A.stable_iters) {
          converged = 1;
          break;
        }
      }
    }
    if (it > A.iters) it = A.iters;
    // Step 10: row argmax; a permutation is the exact assignment optimum.
    // Otherwise the exact assignment, with its arrays in this workgroup's
    // LDS (the iteration's shared buffers are free by now).
    if (!tracked) wg_argmax(Nf, n, np, sigma, nullptr, sh);
    const int is_perm = sh.flag;
    __syncthreads();
    int paths = 0;
    if (!is_perm) {
      char* base = reinterpret_cast<char*>(&sh);
      paths = lap_solve<kBT>(Nf, n, (size_t)np, sigma, nullptr, nullptr, 0,
                             lap_carve(base, n, reinterpret_cast<int*>(base + lap_array_bytes(n))),
                             lsh);
    }
    if (tid == 0) {
      R.outer_iters = it;
      R.sdsn_passes = total;
      R.sdsn_passes_max = pmax;
      R.sdsn_passes_last = plast;
      R.converged = converged;
      R.sdsn_capped = capped;
      R.delta = delta;
      R.gamma = gamma;
      R.is_perm = is_perm;
      R.lap_paths = paths;
    }
    __syncthreads();
  }
  // Objective (eq. 1 without node term) on the unscaled inputs, FP64.
  double acc = 0.0;
  for (size_t t = tid; t < nn; t += kBT) {
    const int k = (int)(t / n), l = (int)(t % n);
    const int sk = sigma[k], sl = sigma[l];
    const bool ok = sk >= 0 && sk < n && sl >= 0 && sl < n;  // else a failed assignment
    acc += ok ? A64[t] * B64[(size_t)sk * n + sl] : __builtin_nan("");
  }
  acc = wg_sum(acc, sh);
  if (tid == 0) R.objective = acc;
}

static_assert(sizeof(Shared) >= (3 * 8 + 3 * 4 + 1 + 4) * kBatchMaxN + 16,
              "the assignment's arrays must fit in the solver's shared buffers");

template <Elem E>
__global__ __launch_bounds__(kBT, 3) void fram_batch_kernel(BatchArgs a) {
  __shared__ Shared sh;
  __shared__ LapShared<kW> lsh;
  __shared__ int s_q;
  while (true) {
    if (threadIdx.x == 0) s_q = atomicAdd(a.next, 1);
    __syncthreads();
    const int q = s_q;
    __syncthreads();
    if (q >= a.count) break;  // every workgroup drains the queue and exits
    const int p = a.order[q];
    solve_pair<E>(a, a.pairs[p], a.res[p], sh, lsh);
  }
}

}  // namespace
}  // namespace fram
