// SDSN (Algorithm 2) with the iterate resident on chip.
//
// The streaming pass in sdsn.hip reads and writes all of X once per SDSN
// iteration, so its time is bounded by HBM.  Here one cooperative launch runs
// every pass of one projection: each workgroup keeps its BM x BM tile of X in
// VGPRs for the whole projection (64 floats per lane at BM = 256 with 1024
// lanes; the n = 4000 iterate, 64 MB, fits in the 128 MB register file of
// 256 CUs).  Per pass only the tile's row/column partial sums (FP64) and its
// total cross the chip: they are written to a ping-pong buffer, a grid-wide
// barrier is taken, and every workgroup then reads the partials of its own
// rows and columns and all tile totals.  Every workgroup evaluates the same
// FP64 gamma = 1^T Y 1 / n - 1 (Sec. 5.2) from the same totals in the same
// order, so all of them leave the pass loop at the same pass.
//
// The same launch optionally finishes Algorithm 1 steps 7-8: with D = Y still
// in registers it updates N <- (1-alpha) N + alpha D, writes the GEMM-type
// copy of N and FP64 partial sums for delta, so X is never written back.
//
// The pass arithmetic and every reduction are those of sdsn.hip (shared in
// sdsn_common.h), so both kernels give bit-identical iterates:
// Y = max(0, fma(s, x, alpha_i + beta_j)) with the symmetric FP64 split of the
// P1 correction (eq. P1_sol).
#include "fram_internal.h"
#include "sdsn_common.h"

namespace fram {
namespace {

// Grid-wide barrier, arrival half: every wave waits for its own global
// stores, then thread 0 makes the workgroup's stores visible device-wide (one
// agent-scope release fence) and publishes the epoch in the workgroup's flag.
__device__ __forceinline__ void barrier_arrive(unsigned long long* flags,
                                               unsigned long long epoch) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(flags + blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Waiting half: every workgroup polls all flags itself (thread t watches
// flag t, relaxed loads), so the barrier costs one cross-chip round trip
// after the last arrival.  Epochs grow monotonically across launches (the
// host passes a fresh 2^24-aligned base per launch), so flags never need
// resetting and a flag already past `epoch` also counts.  Waits are bounded:
// a workgroup that gives up returns false and its caller leaves the pass loop,
// so the grid always drains.  One agent-scope acquire fence follows.
__device__ __forceinline__ bool barrier_wait(unsigned long long* flags, unsigned long long epoch,
                                             int spin_limit, int* s_ok) {
  const int G = gridDim.x;
  int ok = 1;
  for (int t = threadIdx.x; t < G; t += blockDim.x) {
    int spins = 0;
    while (__hip_atomic_load(flags + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > spin_limit) {
        ok = 0;
        break;
      }
    }
    if (!ok) break;
  }
  if (threadIdx.x == 0) *s_ok = 1;
  __syncthreads();
  if (!ok) *s_ok = 0;
  __syncthreads();
  const bool all = *s_ok != 0;
  if (threadIdx.x == 0 && all) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
  return all;
}

template <int BM>
__global__ __launch_bounds__(4 * BM) void sdsn_persistent_kernel(PersistArgs a) {
  using TS = TileShape<BM>;
  constexpr int NT = TS::NT;
  constexpr int LPR = TS::LPR;
  constexpr int RPW = TS::RPW;
  constexpr int STEPS = TS::STEPS;
  __shared__ double s_rowsum[BM];
  __shared__ float s_colred[16][BM];
  __shared__ float s_a[BM];
  __shared__ float s_b[BM];
  __shared__ double s_red[NT / 64];
  __shared__ double s_chain[2][4][BM];
  __shared__ int s_ok;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // Wave index as a scalar: row bounds then stay in SGPRs.
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = a.n, np = a.np, nb = np / BM;
  const int G = gridDim.x;
  int t = blockIdx.x;  // tile index
  if ((G & 7) == 0) t = (t & 7) * (G >> 3) + (t >> 3);  // tile rows share an XCD
  const int bm = t / nb, bn = t % nb;
  const int q = lane / LPR;
  const int cl = (lane % LPR) * 4;
  const int j = bn * BM + cl;
  const bool c0 = j < n, c1 = j + 1 < n, c2 = j + 2 < n, c3 = j + 3 < n;

  // ---- load the tile (rows >= n and columns >= n read as zero) and emit the
  // partials and maximum of the input
  float4 xv[STEPS];
  float lmax = -INFINITY;
  float4 cacc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int stp = 0; stp < STEPS; ++stp) {
    const int rl = w * 16 + stp * RPW + q;
    const int i = bm * BM + rl;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < n) {
      const float* row = &at_u32(a.src, (unsigned)(i * a.ld_src + j));
      // A float4 only where all four columns are inside the matrix: src may
      // have leading dimension n, so a row's tail must not be read past.
      if (a.src_vec && c3) {
        v = *reinterpret_cast<const float4*>(row);
      } else {
        v.x = c0 ? row[0] : 0.f;
        v.y = c1 ? row[1] : 0.f;
        v.z = c2 ? row[2] : 0.f;
        v.w = c3 ? row[3] : 0.f;
      }
      if (c0) lmax = fmaxf(lmax, v.x);
      if (c1) lmax = fmaxf(lmax, v.y);
      if (c2) lmax = fmaxf(lmax, v.z);
      if (c3) lmax = fmaxf(lmax, v.w);
    }
    xv[stp] = v;
    tile_step_sums<BM>(v, rl, s_rowsum, cacc);
  }
  tile_partials<BM>(cacc, s_rowsum, s_colred, s_red, a.p[0].rowp, a.p[0].colp, a.p[0].tot, bm,
                    bn, nb, np);
  {
    const float tm = block_max<NT>(lmax, reinterpret_cast<float*>(s_red));
    if (tid == 0) a.p[0].tmax[bm * nb + bn] = tm;
  }
  unsigned long long epoch = a.epoch_base + 1;
  barrier_arrive(a.flags, epoch);

  int k = 1;
  double gamma = 0.0;
  bool ok = true;
  const double dn = (double)n;
  for (;; ++k) {
    ok = barrier_wait(a.flags, epoch, a.spin_limit, &s_ok);
    if (!ok) break;
    const Partials in = a.p[(k - 1) & 1];
    const Partials out = a.p[k & 1];
    // All reads of the previous pass's partials are issued before any wait:
    // the tile totals, then thread (p, r)'s chains p of row r's and column
    // r's partial sums (combined in a fixed order after the barrier below).
    // The totals decide when every workgroup leaves the loop, so they are
    // read with agent-scope atomic loads, which never hit a stale cache line
    // even if a cache's invalidation were missed: all workgroups must see the
    // same values to take the same decision.
    double part = 0.0;
#pragma unroll 1
    for (int u = tid; u < nb * nb; u += NT)
      part += __hip_atomic_load(&at_u32(in.tot, (unsigned)u), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT);
    float m = -INFINITY;
    if (k == 1)
      for (int u = tid; u < nb * nb; u += NT)
        m = fmaxf(m, __hip_atomic_load(&at_u32(in.tmax, (unsigned)u), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT));
    {
      const int r = tid % BM, p = tid / BM;
      const unsigned ro = (unsigned)(bm * BM + r), co = (unsigned)(bn * BM + r);
      auto ldr = [&](int b) { return at_u32(in.rowp, (unsigned)(b * np) + ro); };
      auto ldc = [&](int b) { return at_u32(in.colp, (unsigned)(b * np) + co); };
      s_chain[0][p][r] = chain_sum(ldr, nb, p);
      s_chain[1][p][r] = chain_sum(ldc, nb, p);
    }
    const double S = block_sum<NT>(part, s_red);
    float s = 1.0f;
    if (k >= 2) {
      gamma = S / dn - 1.0;
      if (gamma <= a.gamma_tol || k > a.max_passes) break;
    } else {
      m = block_max<NT>(m, reinterpret_cast<float*>(s_red));
      s = (m > 0.0f) ? (float)(a.theta / (2.0 * (double)m)) : 0.0f;
    }
    const double sd = (double)s;
    const double half = 0.5 / dn + 0.5 * sd * S / (dn * dn);
    if (tid < BM) {
      const double ri = combine4(s_chain[0][0][tid], s_chain[0][1][tid], s_chain[0][2][tid],
                                 s_chain[0][3][tid]);
      const double cj = combine4(s_chain[1][0][tid], s_chain[1][1][tid], s_chain[1][2][tid],
                                 s_chain[1][3][tid]);
      s_a[tid] = (float)(half - sd * ri / dn);
      s_b[tid] = (float)(half - sd * cj / dn);
    }
    __syncthreads();
    const float4 bt = make_float4(s_b[cl], s_b[cl + 1], s_b[cl + 2], s_b[cl + 3]);
    cacc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int stp = 0; stp < STEPS; ++stp) {
      const int rl = w * 16 + stp * RPW + q;
      const float ai = s_a[rl];
      float4 y = make_float4(0.f, 0.f, 0.f, 0.f);
      if (bm * BM + rl < n) {
        const float4 x = xv[stp];
        y.x = c0 ? fmaxf(0.0f, fmaf(s, x.x, ai + bt.x)) : 0.0f;
        y.y = c1 ? fmaxf(0.0f, fmaf(s, x.y, ai + bt.y)) : 0.0f;
        y.z = c2 ? fmaxf(0.0f, fmaf(s, x.z, ai + bt.z)) : 0.0f;
        y.w = c3 ? fmaxf(0.0f, fmaf(s, x.w, ai + bt.w)) : 0.0f;
      }
      xv[stp] = y;
      tile_step_sums<BM>(y, rl, s_rowsum, cacc);
    }
    tile_partials<BM>(cacc, s_rowsum, s_colred, s_red, out.rowp, out.colp, out.tot, bm, bn, nb,
                      np);
    ++epoch;
    barrier_arrive(a.flags, epoch);
  }
  if (!ok) {
    if (tid == 0) atomicOr(&a.st->invalid, 8);
    return;
  }
  const int passes = k - 1;

  if (a.dst != nullptr) {
#pragma unroll
    for (int stp = 0; stp < STEPS; ++stp) {
      const int i = bm * BM + w * 16 + stp * RPW + q;
      if (i < n) *reinterpret_cast<float4*>(&at_u32(a.dst, (unsigned)(i * np + j))) = xv[stp];
    }
  }
  if (a.N != nullptr) {
    // Algorithm 1 steps 7-8 on this tile: N <- (1-alpha) N + alpha D.
    const float alpha = a.alpha, c1a = 1.0f - a.alpha;
    double num = 0.0, den = 0.0;
    // Fully unrolled (a runtime index into xv would force it out of VGPRs),
    // in groups of four rows with a scheduling barrier between groups so that
    // the loads of N do not all become live at once next to the tile.
#pragma unroll
    for (int stp = 0; stp < STEPS; ++stp) {
      if ((stp & 3) == 0) __builtin_amdgcn_sched_barrier(0);
      const int i = bm * BM + w * 16 + stp * RPW + q;
      if (i >= n) continue;
      const unsigned idx = (unsigned)(i * np + j);
      float4& nref = *reinterpret_cast<float4*>(&at_u32(a.N, idx));
      const float4 o = nref;
      const float4 d = xv[stp];
      float4 nn;
      nn.x = fmaf(alpha, d.x, c1a * o.x);
      nn.y = fmaf(alpha, d.y, c1a * o.y);
      nn.z = fmaf(alpha, d.z, c1a * o.z);
      nn.w = fmaf(alpha, d.w, c1a * o.w);
      nref = nn;
      if (a.nlp_kind == 1) {
        __bf16* o16 = &at_u32(reinterpret_cast<__bf16*>(a.Nlp), idx);
        o16[0] = (__bf16)nn.x;
        o16[1] = (__bf16)nn.y;
        o16[2] = (__bf16)nn.z;
        o16[3] = (__bf16)nn.w;
      } else if (a.nlp_kind == 2) {
        _Float16* o16 = &at_u32(reinterpret_cast<_Float16*>(a.Nlp), idx);
        o16[0] = (_Float16)nn.x;
        o16[1] = (_Float16)nn.y;
        o16[2] = (_Float16)nn.z;
        o16[3] = (_Float16)nn.w;
      }
      const double ex = (double)nn.x - (double)o.x, ey = (double)nn.y - (double)o.y;
      const double ez = (double)nn.z - (double)o.z, ew = (double)nn.w - (double)o.w;
      num += (ex * ex + ey * ey) + (ez * ez + ew * ew);
      den += ((double)nn.x * nn.x + (double)nn.y * nn.y) +
             ((double)nn.z * nn.z + (double)nn.w * nn.w);
    }
    num = block_sum<NT>(num, s_red);
    den = block_sum<NT>(den, s_red);
    if (tid == 0) {
      a.dpart[2 * (bm * nb + bn)] = num;
      a.dpart[2 * (bm * nb + bn) + 1] = den;
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    DevState* st = a.st;
    st->done = 1;
    st->passes = passes;
    st->gamma = gamma;
    st->total_passes += passes;
    if (passes > st->max_passes) st->max_passes = passes;
    if (passes >= a.max_passes && !(gamma <= a.gamma_tol)) st->capped = 1;
  }
}

template <int BM>
hipError_t launch_bm(const PersistArgs& a, hipStream_t s) {
  const int nb = a.np / BM;
  void* args[] = {const_cast<PersistArgs*>(&a)};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&sdsn_persistent_kernel<BM>),
                                    dim3(nb * nb), dim3(4 * BM), args, 0, s);
}

template <int BM>
bool fits_bm(int device, int nblocks) {
  int per_cu = 0, cus = 0, coop = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess ||
      !coop)
    return false;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return false;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(&sdsn_persistent_kernel<BM>), 4 * BM, 0) !=
      hipSuccess)
    return false;
  return (long)per_cu * cus >= nblocks;
}

}  // namespace

bool sdsn_persistent_fits(int device, int bm, int np) {
  const int nb = np / bm;
  switch (bm) {
    case 64:
      return fits_bm<64>(device, nb * nb);
    case 128:
      return fits_bm<128>(device, nb * nb);
    case 256:
      return fits_bm<256>(device, nb * nb);
  }
  return false;
}

hipError_t launch_sdsn_persistent(int bm, const PersistArgs& a, hipStream_t s) {
  if (a.np % bm != 0 || a.n > a.np || a.n < 1) return hipErrorInvalidValue;
  switch (bm) {
    case 64:
      return launch_bm<64>(a, s);
    case 128:
      return launch_bm<128>(a, s);
    case 256:
      return launch_bm<256>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace fram
