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
// The pass arithmetic is the one of sdsn.hip: Y = max(0, fma(s, x, alpha_i +
// beta_j)) with the symmetric FP64 split of the P1 correction (eq. P1_sol).
#include "fram_internal.h"
#include "sdsn_common.h"

namespace fram {
namespace {

// Grid-wide barrier without a contended counter.  Every wave first waits for
// its own outstanding global stores; thread 0 then makes the workgroup's
// stores visible device-wide (one agent-scope release fence) and publishes
// the barrier's epoch in the workgroup's own flag.  Workgroup 0 waits for all
// flags and publishes the epoch in a release flag that every workgroup waits
// for.  Polling uses relaxed loads; one agent-scope acquire fence follows a
// successful wait.  Epochs grow monotonically across launches (the host passes
// a fresh 2^24-aligned base per launch), so flags never need resetting.
// Waits are bounded: a workgroup that gives up returns false and the caller
// leaves the pass loop, so the grid always drains.
__device__ bool grid_barrier(unsigned long long* flags, unsigned long long epoch, int spin_limit) {
  __shared__ int s_ok;
  const int G = gridDim.x;
  unsigned long long* release = flags + G;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(flags + blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_ok = 1;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < G; t += blockDim.x) {
      int spins = 0;
      while (__hip_atomic_load(flags + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > spin_limit) {
          s_ok = 0;
          break;
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0 && s_ok) {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
      __hip_atomic_store(release, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (threadIdx.x == 0 && s_ok) {
    int spins = 0;
    while (__hip_atomic_load(release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > spin_limit) {
        s_ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return s_ok != 0;
}

__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float ld_agent(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Row/column partials of the tile values in xv into set `out` (FP64 from
// per-lane FP32 sums of at most 16 elements, fixed order).  The next grid
// barrier makes these stores visible to the other workgroups.
template <int BM>
__device__ __forceinline__ void emit_partials(const float4 (&xv)[16 / (64 / (BM / 4))],
                                              const Partials& out,
                                              float (*s_rowred)[BM / 4 + 1], float (*s_colred)[BM],
                                              double* s_red, int bm, int bn, int nb, int np) {
  constexpr int NT = 4 * BM;
  constexpr int LPR = BM / 4;
  constexpr int RPW = 64 / LPR;
  constexpr int STEPS = 16 / RPW;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // Wave index as a scalar: row bounds then stay in SGPRs.
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane / LPR;
  const int lc = lane % LPR;
  const int cl = lc * 4;
  float4 cacc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int stp = 0; stp < STEPS; ++stp) {
    const float4 y = xv[stp];
    s_rowred[w * 16 + stp * RPW + q][lc] = (y.x + y.y) + (y.z + y.w);
    cacc.x += y.x;
    cacc.y += y.y;
    cacc.z += y.z;
    cacc.w += y.w;
  }
  *reinterpret_cast<float4*>(&s_colred[w * RPW + q][cl]) = cacc;
  __syncthreads();
  const int r = tid >> 2, p = tid & 3;
  double v = 0.0;
#pragma unroll
  for (int u = 0; u < LPR / 4; ++u) v += (double)s_rowred[r][p * (LPR / 4) + u];
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  if (p == 0) out.rowp[(size_t)bn * np + bm * BM + r] = v;
  const double rowsum = (p == 0) ? v : 0.0;
  double cv = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u) cv += (double)s_colred[p * 4 + u][r];
  cv += __shfl_xor(cv, 1);
  cv += __shfl_xor(cv, 2);
  if (p == 0) out.colp[(size_t)bm * np + bn * BM + r] = cv;
  const double tt = block_sum<NT>(rowsum, s_red);
  if (tid == 0) out.tot[bm * nb + bn] = tt;
}

template <int BM>
__global__ __launch_bounds__(4 * BM) void sdsn_persistent_kernel(PersistArgs a) {
  constexpr int NT = 4 * BM;
  constexpr int LPR = BM / 4;
  constexpr int RPW = 64 / LPR;
  constexpr int STEPS = 16 / RPW;
  __shared__ float s_rowred[BM][LPR + 1];
  __shared__ float s_colred[16][BM];
  __shared__ float s_a[BM];
  __shared__ float s_b[BM];
  __shared__ double s_red[NT];
  __shared__ double s_chain[2][4][BM];

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
  const int lc = lane % LPR;
  const int cl = lc * 4;
  const int j = bn * BM + cl;
  const bool c0 = j < n, c1 = j + 1 < n, c2 = j + 2 < n, c3 = j + 3 < n;

  // ---- load the tile (rows >= n and columns >= n read as zero)
  float4 xv[STEPS];
  float lmax = -INFINITY;
#pragma unroll
  for (int stp = 0; stp < STEPS; ++stp) {
    const int i = bm * BM + w * 16 + stp * RPW + q;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < n) {
      const float* row = a.src + (size_t)i * a.ld_src + j;
      if (a.src_vec) {
        v = *reinterpret_cast<const float4*>(row);
        v.x = c0 ? v.x : 0.f;
        v.y = c1 ? v.y : 0.f;
        v.z = c2 ? v.z : 0.f;
        v.w = c3 ? v.w : 0.f;
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
  }

  emit_partials<BM>(xv, a.p[0], s_rowred, s_colred, s_red, bm, bn, nb, np);
  {
    const float tm = block_max<NT>(lmax, reinterpret_cast<float*>(s_red));
    if (tid == 0) a.p[0].tmax[bm * nb + bn] = tm;
  }
  unsigned long long epoch = a.epoch_base + 1;
  bool ok = grid_barrier(a.flags, epoch, a.spin_limit);

  int k = 1;
  double gamma = 0.0;
  const double dn = (double)n;
  for (; ok; ++k) {
    const Partials in = a.p[(k - 1) & 1];
    const Partials out = a.p[k & 1];
    double part = 0.0;
#pragma unroll 1
    for (int u = tid; u < nb * nb; u += NT) part += ld_agent(in.tot + u);
    const double S = block_sum<NT>(part, s_red);
    float s = 1.0f;
    if (k >= 2) {
      gamma = S / dn - 1.0;
      if (gamma <= a.gamma_tol || k > a.max_passes) break;
    } else {
      float m = -INFINITY;
      for (int u = tid; u < nb * nb; u += NT) m = fmaxf(m, ld_agent(in.tmax + u));
      m = block_max<NT>(m, reinterpret_cast<float*>(s_red));
      s = (m > 0.0f) ? (float)(a.theta / (2.0 * (double)m)) : 0.0f;
    }
    const double sd = (double)s;
    const double half = 0.5 / dn + 0.5 * sd * S / (dn * dn);
    {
      // Thread (p, r) forms chain p of row r's and column r's partial sums;
      // the four chains are then combined in a fixed order.
      const int r = tid % BM, p = tid / BM;
      const double* rp = in.rowp + bm * BM + r;
      const double* cp = in.colp + bn * BM + r;
      auto ldr = [&](int b) { return ld_agent(rp + (size_t)b * np); };
      auto ldc = [&](int b) { return ld_agent(cp + (size_t)b * np); };
      s_chain[0][p][r] = chain_sum(ldr, nb, p);
      s_chain[1][p][r] = chain_sum(ldc, nb, p);
      __syncthreads();
      if (tid < BM) {
        const double ri = combine4(s_chain[0][0][tid], s_chain[0][1][tid], s_chain[0][2][tid],
                                   s_chain[0][3][tid]);
        const double cj = combine4(s_chain[1][0][tid], s_chain[1][1][tid], s_chain[1][2][tid],
                                   s_chain[1][3][tid]);
        s_a[tid] = (float)(half - sd * ri / dn);
        s_b[tid] = (float)(half - sd * cj / dn);
      }
    }
    __syncthreads();
    const float4 bt = make_float4(s_b[cl], s_b[cl + 1], s_b[cl + 2], s_b[cl + 3]);
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
    }
    emit_partials<BM>(xv, out, s_rowred, s_colred, s_red, bm, bn, nb, np);
    ++epoch;
    ok = grid_barrier(a.flags, epoch, a.spin_limit);
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
      if (i < n) *reinterpret_cast<float4*>(a.dst + (size_t)i * np + j) = xv[stp];
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
      const size_t idx = (size_t)i * np + j;
      const float4 o = *reinterpret_cast<const float4*>(a.N + idx);
      const float4 d = xv[stp];
      float4 nn;
      nn.x = fmaf(alpha, d.x, c1a * o.x);
      nn.y = fmaf(alpha, d.y, c1a * o.y);
      nn.z = fmaf(alpha, d.z, c1a * o.z);
      nn.w = fmaf(alpha, d.w, c1a * o.w);
      *reinterpret_cast<float4*>(a.N + idx) = nn;
      if (a.nlp_kind == 1) {
        __bf16* o16 = reinterpret_cast<__bf16*>(a.Nlp) + idx;
        o16[0] = (__bf16)nn.x;
        o16[1] = (__bf16)nn.y;
        o16[2] = (__bf16)nn.z;
        o16[3] = (__bf16)nn.w;
      } else if (a.nlp_kind == 2) {
        _Float16* o16 = reinterpret_cast<_Float16*>(a.Nlp) + idx;
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
