// SDSN (Algorithm 2) as one fused, memory-bound pass per iteration.
//
// One pass maps its input X to
//     Y = P2(P1(s X)),
//     P1(Z)_ij = Z_ij + 1/n + (1^T Z 1)/n^2 - (Z 1)_i/n - (1^T Z)_j/n   (eq. P1_sol)
//     P2(Z)    = max(0, Z)                                              (Sec. 5.1)
// with s = theta / (2 max X) on the first pass (Alg. 2, first line) and 1
// afterwards.  Since the row sums r, column sums c and total S of the input
// are all P1 needs, each pass also produces r, c and S of its output, so the
// next pass can start immediately: the row and column sums are written as
// per-tile FP64 partials (fixed order, no atomics), and the stopping measure
// gamma = 1^T Y 1 / n - 1 (Sec. 5.2, App. B.1) of a pass output is evaluated
// in FP64 at the start of the next pass.  A pass that finds gamma <= gamma_tol
// marks the projection done and leaves X untouched, so a host loop may launch
// passes in chunks and read the flag once per chunk.
//
// Precision.  The correction is split symmetrically,
//     1/n + sS/n^2 - s r_i/n - s c_j/n = alpha_i + beta_j,
//     alpha_i = 1/(2n) + sS/(2n^2) - s r_i/n,  beta_j = 1/(2n) + sS/(2n^2) - s c_j/n,
// and formed in FP64 from FP64 sums.  Near convergence (s = 1, r, c ~ 1,
// S ~ n) both terms are O(gamma/n) and keep full FP32 relative precision, so
// Y = max(0, fma(s, x, alpha_i + beta_j)) rounds once at the size of x.
//
// Tiles are BM x BM with 4*BM threads: each wave streams 16 rows of the tile,
// each lane a float4 of columns, so every global access of a wave is one or
// more contiguous 1 KB runs.  Row partials are summed in FP64 across the lanes
// of a row by a transposing pairwise tree over all of the wave's rows at once
// (lane swaps and DPP); column partials stay in registers until the end of the
// tile and are then summed in FP64 through LDS.
#include "fram_internal.h"
#include "sdsn_common.h"

namespace fram {
namespace {

struct TileArgs {
  const float* src;  // input matrix
  int ld_src;
  float* dst;        // output matrix (may equal src), leading dimension np
  int n, np;
  Partials in, out;
  DevState* st;
  int k, max_passes;
  double theta, gamma_tol;
  double fixed_scale;  // > 0: first-pass scale s itself, instead of theta / (2 max X)
};

// PASS = false: statistics of src (and optional padded copy into dst).
// PASS = true : one SDSN pass, in place on dst (== src, ld np); returns true
// when the projection is complete (this pass found it done or marked it), the
// same value in every thread of the workgroup.
// WHOLE (passes only, for a matrix that is one padded tile): every row of the
// wave is read before the first is written, so a pass costs one memory round
// trip instead of one per row; rows and columns past n are read (zero
// padding) and written back as zeros.
// Tile (bm, bn) of an nb x nb tile grid.
template <int BM, bool PASS, bool WHOLE = false>
__device__ __forceinline__ bool tile_body(const TileArgs& a, int bm, int bn, int nb) {
  constexpr int NT = TileShape<BM>::NT;
  constexpr int LPR = TileShape<BM>::LPR;      // lanes per tile row
  constexpr int RPW = TileShape<BM>::RPW;      // tile rows per wave step
  constexpr int STEPS = TileShape<BM>::STEPS;  // each wave covers 16 rows
  __shared__ double s_rowsum[BM];
  __shared__ float s_colred[16][BM];
  __shared__ float s_a[BM];
  __shared__ float s_b[BM];
  __shared__ double s_red[NT];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // Wave index as a scalar: row bounds then stay in SGPRs.
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = a.n, np = a.np;
  DevState* st = a.st;

  float s = 1.0f;
  if (PASS) {
    // Every read of the pass's scalar inputs is issued before the first
    // barrier: the done flag (one thread, so the whole workgroup takes the
    // same branch even if another workgroup sets it meanwhile), the tile
    // totals, and, per thread (p, r), chain p of row r's and of column r's
    // partial sums (combined in a fixed order below, so the result is that
    // of summing each chain and combining them in sequence).
    __shared__ int s_done;
    __shared__ double s_chain[2][4][BM];
    const int done = (tid == 0)
        ? __hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    double part = 0.0;
    float m = -INFINITY;
    double rsum, csum;
    const int r = tid % BM, p = tid / BM;
    const double* rp = a.in.rowp + bm * BM + r;
    const double* cp = a.in.colp + bn * BM + r;
    auto ldr = [&](int b) { return rp[(size_t)b * np]; };
    auto ldc = [&](int b) { return cp[(size_t)b * np]; };
    if (nb <= 16) {
      // Then nb * nb <= NT: one total (and first-pass maximum) per thread,
      // read with the chains before any of them is used, so the whole
      // prologue waits for memory once.  The maxima buffer is valid on every
      // pass; its values are used on the first.
      const bool has_t = tid < nb * nb;
      const int t = has_t ? tid : 0;
      const double tv = a.in.tot[t];
      const float mv = a.in.tmax[t];
      chain_sum_pair16(ldr, ldc, nb, p, rsum, csum);
      part = has_t ? part + tv : part;
      m = (has_t && a.k == 1) ? fmaxf(m, mv) : m;
    } else {
      for (int t = tid; t < nb * nb; t += NT) part += a.in.tot[t];
      if (a.k == 1)
        for (int t = tid; t < nb * nb; t += NT) m = fmaxf(m, a.in.tmax[t]);
      rsum = chain_sum(ldr, nb, p);
      csum = chain_sum(ldc, nb, p);
    }
    s_chain[0][p][r] = rsum;
    s_chain[1][p][r] = csum;
    if (tid == 0) s_done = done;
    const double S = block_sum<NT>(part, s_red);  // its barriers publish s_done, s_chain
    if (s_done) return true;
    if (a.k >= 2) {
      const double gamma_in = S / n - 1.0;
      if (gamma_in <= a.gamma_tol || a.k > a.max_passes) {
        if (bm == 0 && bn == 0 && tid == 0) {
          st->done = 1;
          st->passes = a.k - 1;
          st->gamma = gamma_in;
        }
        return true;
      }
    } else {
      m = block_max<NT>(m, reinterpret_cast<float*>(s_red));
      s = (a.fixed_scale > 0.0) ? (float)a.fixed_scale
                                : ((m > 0.0f) ? (float)(a.theta / (2.0 * (double)m)) : 0.0f);
    }
    const double sd = (double)s;
    const double dn = (double)n;
    const double half = 0.5 / dn + 0.5 * sd * S / (dn * dn);
    if (tid < BM) {
      const double ri = combine4(s_chain[0][0][tid], s_chain[0][1][tid], s_chain[0][2][tid],
                                 s_chain[0][3][tid]);
      const double cj = combine4(s_chain[1][0][tid], s_chain[1][1][tid], s_chain[1][2][tid],
                                 s_chain[1][3][tid]);
      // Rows and columns past n get -inf, so their entries (zero) map to
      // max(0, -inf) = 0 without a test per entry.
      s_a[tid] = (bm * BM + tid < n) ? (float)(half - sd * ri / dn) : -INFINITY;
      s_b[tid] = (bn * BM + tid < n) ? (float)(half - sd * cj / dn) : -INFINITY;
    }
    __syncthreads();
  } else {
    if (bm == 0 && bn == 0 && tid == 0) {
      st->done = 0;
      st->passes = 0;
    }
  }

  const int q = lane / LPR;
  const int lc = lane % LPR;
  const int cl = lc * 4;
  const int j = bn * BM + cl;
  float4 bt = make_float4(0.f, 0.f, 0.f, 0.f);
  if (PASS) bt = make_float4(s_b[cl], s_b[cl + 1], s_b[cl + 2], s_b[cl + 3]);
  float4 cacc = make_float4(0.f, 0.f, 0.f, 0.f);
  RowSums<BM> rows;
  float lmax = -INFINITY;
  const bool c0 = j < n, c1 = j + 1 < n, c2 = j + 2 < n, c3 = j + 3 < n;

  if constexpr (PASS && WHOLE) {
    float4 xv[STEPS];
#pragma unroll
    for (int stp = 0; stp < STEPS; ++stp)
      xv[stp] = *reinterpret_cast<const float4*>(a.dst + (size_t)(w * 16 + stp * RPW + q) * np + j);
#pragma unroll
    for (int stp = 0; stp < STEPS; ++stp) {
      const int rl = w * 16 + stp * RPW + q;
      const float ai = s_a[rl];
      const float4 x = xv[stp];
      float4 y;
      y.x = fmaxf(0.0f, fmaf(s, x.x, ai + bt.x));
      y.y = fmaxf(0.0f, fmaf(s, x.y, ai + bt.y));
      y.z = fmaxf(0.0f, fmaf(s, x.z, ai + bt.z));
      y.w = fmaxf(0.0f, fmaf(s, x.w, ai + bt.w));
      *reinterpret_cast<float4*>(a.dst + (size_t)rl * np + j) = y;
      tile_step_sums<BM>(y, stp, rows, cacc);
    }
  } else {
#pragma unroll
  for (int stp = 0; stp < STEPS; ++stp) {
    const int rl = w * 16 + stp * RPW + q;
    const int i = bm * BM + rl;
    float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
    // In a pass, lanes whose four columns all lie past n (the padding of the
    // last column tile, zero since the matrix was written) neither read nor
    // write: the pass would only store zeros there again.
    if (i < n && (!PASS || c0)) {
      if (PASS) {
        float4* row = reinterpret_cast<float4*>(a.dst + (size_t)i * np + j);
        const float4 x = *row;
        const float ai = s_a[rl];
        y.x = fmaxf(0.0f, fmaf(s, x.x, ai + bt.x));
        y.y = fmaxf(0.0f, fmaf(s, x.y, ai + bt.y));
        y.z = fmaxf(0.0f, fmaf(s, x.z, ai + bt.z));
        y.w = fmaxf(0.0f, fmaf(s, x.w, ai + bt.w));
        *row = y;
      } else {
        const float* row = a.src + (size_t)i * a.ld_src + j;
        y.x = c0 ? row[0] : 0.0f;
        y.y = c1 ? row[1] : 0.0f;
        y.z = c2 ? row[2] : 0.0f;
        y.w = c3 ? row[3] : 0.0f;
        if (c0) lmax = fmaxf(lmax, y.x);
        if (c1) lmax = fmaxf(lmax, y.y);
        if (c2) lmax = fmaxf(lmax, y.z);
        if (c3) lmax = fmaxf(lmax, y.w);
        if (a.dst != nullptr && a.dst != a.src)
          *reinterpret_cast<float4*>(a.dst + (size_t)i * np + j) = y;
      }
    } else if (!PASS && a.dst != nullptr && a.dst != a.src) {
      *reinterpret_cast<float4*>(a.dst + (size_t)i * np + j) = y;
    }
    tile_step_sums<BM>(y, stp, rows, cacc);
  }
  }
  rows.finish(w, s_rowsum);
  tile_partials<BM>(cacc, s_rowsum, s_colred, s_red, a.out.rowp, a.out.colp, a.out.tot, bm, bn,
                    nb, np);
  if (!PASS) {
    const float tm = block_max<NT>(lmax, reinterpret_cast<float*>(s_red));
    if (tid == 0) a.out.tmax[bm * nb + bn] = tm;
  }
  return false;
}

template <int BM, bool PASS>
__global__ __launch_bounds__(4 * BM) void tile_kernel(TileArgs a) {
  (void)tile_body<BM, PASS>(a, blockIdx.y, blockIdx.x, gridDim.x);
}

// Passes a.k .. k_last of a projection whose matrix is a single tile, in one
// workgroup: pass k + 1 reads the partial sums that pass k wrote, which the
// workgroup barrier between them makes visible, so no launch (and no host
// round trip) separates the passes.  Stops at the pass that completes the
// projection, exactly where the per-pass launches would.
template <int BM>
__global__ __launch_bounds__(4 * BM) void tile_chunk_kernel(TileArgs a, Partials p0, Partials p1,
                                                            int k_last) {
  for (int k = a.k; k <= k_last; ++k) {
    a.k = k;
    a.in = ((k - 1) & 1) ? p1 : p0;
    a.out = (k & 1) ? p1 : p0;
    // Whole-tile loads pay off while the wave's rows fit in registers next to
    // everything else (BM <= 128); at 256 they spill.
    if (tile_body<BM, true, (BM <= 128)>(a, 0, 0, 1)) break;
    __syncthreads();
  }
}

// One projection per job (blockIdx.x), each a single tile: the statistics
// pass of tile_kernel<BM, false> (dst = nullptr) and then every pass of
// tile_chunk_kernel, in one workgroup -- the same iterates as those two
// launches.
template <int BM>
__global__ __launch_bounds__(4 * BM) void sdsn_group_kernel(const SdsnJob* __restrict__ jobs,
                                                            int max_passes, double theta,
                                                            double gamma_tol) {
  const SdsnJob j = jobs[blockIdx.x];
  TileArgs a{};
  a.src = j.X;
  a.ld_src = j.np;
  a.dst = nullptr;
  a.n = j.n;
  a.np = j.np;
  a.out = j.p0;
  a.st = j.st;
  (void)tile_body<BM, false>(a, 0, 0, 1);
  __syncthreads();
  a.dst = j.X;
  a.max_passes = max_passes;
  a.theta = theta;
  a.gamma_tol = gamma_tol;
  const int k_last = max_passes + 1;
  for (int k = 1; k <= k_last; ++k) {
    a.k = k;
    a.in = ((k - 1) & 1) ? j.p1 : j.p0;
    a.out = (k & 1) ? j.p1 : j.p0;
    if (tile_body<BM, true, (BM <= 128)>(a, 0, 0, 1)) break;
    __syncthreads();
  }
}

template <bool PASS>
hipError_t launch_tile(int bm, const TileArgs& a, hipStream_t s) {
  const int nb = a.np / bm;
  dim3 grid(nb, nb);
  switch (bm) {
    case 64:
      tile_kernel<64, PASS><<<grid, dim3(256), 0, s>>>(a);
      break;
    case 128:
      tile_kernel<128, PASS><<<grid, dim3(512), 0, s>>>(a);
      break;
    case 256:
      tile_kernel<256, PASS><<<grid, dim3(1024), 0, s>>>(a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_tile_stats(int bm, const float* src, int ld_src, float* dst, int n, int np,
                             Partials out, DevState* st, hipStream_t s) {
  if (np % bm != 0 || n > np || n < 1) return hipErrorInvalidValue;
  TileArgs a{};
  a.src = src;
  a.ld_src = ld_src;
  a.dst = dst;
  a.n = n;
  a.np = np;
  a.out = out;
  a.st = st;
  return launch_tile<false>(bm, a, s);
}

hipError_t launch_sdsn_chunk(int bm, float* X, int n, int np, Partials p0, Partials p1,
                             DevState* st, int k_first, int k_last, int max_passes, double theta,
                             double gamma_tol, hipStream_t s, double fixed_scale) {
  if (np != bm || n > np || n < 1 || k_first < 1 || k_last < k_first) return hipErrorInvalidValue;
  TileArgs a{};
  a.src = X;
  a.ld_src = np;
  a.dst = X;
  a.n = n;
  a.np = np;
  a.st = st;
  a.k = k_first;
  a.max_passes = max_passes;
  a.theta = theta;
  a.gamma_tol = gamma_tol;
  a.fixed_scale = fixed_scale;
  const dim3 one(1, 1);
  switch (bm) {
    case 64:
      tile_chunk_kernel<64><<<one, dim3(256), 0, s>>>(a, p0, p1, k_last);
      break;
    case 128:
      tile_chunk_kernel<128><<<one, dim3(512), 0, s>>>(a, p0, p1, k_last);
      break;
    case 256:
      tile_chunk_kernel<256><<<one, dim3(1024), 0, s>>>(a, p0, p1, k_last);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sdsn_group(int bm, const SdsnJob* jobs, int count, int max_passes,
                             double theta, double gamma_tol, hipStream_t s) {
  if (count < 1) return hipSuccess;
  switch (bm) {
    case 64:
      sdsn_group_kernel<64><<<count, 256, 0, s>>>(jobs, max_passes, theta, gamma_tol);
      break;
    case 128:
      sdsn_group_kernel<128><<<count, 512, 0, s>>>(jobs, max_passes, theta, gamma_tol);
      break;
    case 256:
      sdsn_group_kernel<256><<<count, 1024, 0, s>>>(jobs, max_passes, theta, gamma_tol);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sdsn_pass(int bm, float* X, int n, int np, Partials in, Partials out,
                            DevState* st, int k, int max_passes, double theta,
                            double gamma_tol, hipStream_t s, double fixed_scale) {
  if (np % bm != 0 || n > np || n < 1 || k < 1) return hipErrorInvalidValue;
  TileArgs a{};
  a.src = X;
  a.ld_src = np;
  a.dst = X;
  a.n = n;
  a.np = np;
  a.in = in;
  a.out = out;
  a.st = st;
  a.k = k;
  a.max_passes = max_passes;
  a.theta = theta;
  a.gamma_tol = gamma_tol;
  a.fixed_scale = fixed_scale;
  return launch_tile<true>(bm, a, s);
}

}  // namespace fram
