// SDSN (Algorithm 2) with the iterate resident on chip.
//
// The streaming pass in sdsn.hip reads and writes all of X once per SDSN
// iteration, so its time is bounded by HBM.  Here one launch runs every pass
// of one projection: each workgroup keeps its BM x BM tile of X in VGPRs for
// the whole projection (64 floats per lane at BM = 256 with 1024 lanes; the
// n = 4000 iterate, 64 MB, fits in the 128 MB register file of 256 CUs).  Per
// pass only the tile's row/column partial sums (FP64) and its total cross the
// chip: they are written to a ping-pong buffer, the workgroups meet at a
// grid-wide barrier, and every workgroup then reads the partials of its own
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
//
// Co-residency.  A workgroup that waits at the barrier holds its compute
// unit, so the launch makes progress only if all of its workgroups are
// resident at once (and stay scheduled).  Three rules make a wait that can
// never end impossible, and a launch that cannot complete harmless:
//  * roll call: every workgroup first checks in and waits, for a bounded time,
//    until the whole grid has; if it has not, every workgroup leaves before
//    touching any data;
//  * every later wait is bounded too; a timeout (for instance while the queue
//    of the launch is preempted) aborts the whole grid.  Every workgroup takes
//    the same decision at each wait (see wait_until), and X, D and N are
//    written only after the last pass, so an aborted launch leaves them as
//    they were.  Either way the state records why, and the caller runs the
//    streaming passes on the untouched input;
//  * the host admits a launch only while the grids that may still run and
//    this one fit on the device together (a compute-unit budget across every
//    stream of the process), so such grids never compete for compute units;
//    other kernels only delay a roll call, since they never wait for these.
//
// Barrier.  Arrival is counted per group of workgroups (blockIdx mod 8: the
// XCD the hardware dispatches it to), and the last arrival of a group bumps
// one release counter that every workgroup polls, so each pass costs a few
// atomics per group and one poll target instead of all-to-all flags
// (measured on MI355X with 256 workgroups, barrier plus the partial-sum
// exchange: 4.9 us per pass, against 9.2 us with one counter for all).  The
// counters live in a per-context block that the host zeroes before each
// launch (stream-ordered), and only grow within a launch.
#include "fram_internal.h"
#include "sdsn_common.h"

#ifndef SDSN_ONCHIP_REG_STEPS
#define SDSN_ONCHIP_REG_STEPS 14
#endif

namespace fram {
namespace {

// Fields of the synchronisation block, each in its own 128-byte line.
constexpr int kLine = 32;  // unsigned ints per line
__device__ __forceinline__ unsigned* sync_group(unsigned* sy, int g) { return sy + g * kLine; }
__device__ __forceinline__ unsigned* sync_release(unsigned* sy) { return sy + 8 * kLine; }
__device__ __forceinline__ unsigned* sync_roll(unsigned* sy) { return sy + 9 * kLine; }

__device__ __forceinline__ unsigned ld_agent(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Data that crosses the chip within the launch (partials, totals, maxima) is
// stored and loaded with agent-scope atomics: the stores write through to the
// device-coherent level and the loads read from it, so no cache write-back or
// invalidation is needed around the barrier (measured on MI355X: 4.9 us per
// pass with 256 workgroups, against 9.7 us with a release/acquire fence pair
// around plain accesses).
struct CoherentStore {
  template <typename T>
  __device__ __forceinline__ void operator()(T* p, T v) const {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};
template <typename T>
__device__ __forceinline__ T ld_coherent(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The counters that waits poll (roll call, release) carry an abort bit.
constexpr unsigned kAbortBit = 0x80000000u;

// Thread 0 waits until the count in *p reaches `target` or the abort bit is
// set.  If `limit` wall-clock ticks pass first, it sets the abort bit, with a
// compare-and-swap that succeeds only while the count is still short of the
// target: so every workgroup decides the same way (all pass, or all see the
// abort; a count completed before the abort is never revoked).  The bit stays
// set, so every later wait on *p fails too.  The result is the same in every
// thread of the workgroup.
__device__ bool wait_until(unsigned* p, unsigned target, long long limit, int* s_ok) {
  if (threadIdx.x == 0) {
    int ok = 1;
    const long long t0 = wall_clock64();
    while (true) {
      const unsigned v = ld_agent(p);
      if (v & kAbortBit) {
        ok = 0;
        break;
      }
      if (v >= target) break;
      if (wall_clock64() - t0 > limit) {
        unsigned expect = v;
        if (__hip_atomic_compare_exchange_strong(p, &expect, v | kAbortBit, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
          ok = 0;
          break;
        }
        continue;  // the count moved meanwhile: look again
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *s_ok = ok;
  }
  __syncthreads();
  return *s_ok != 0;
}

// Barrier number `epoch` (1, 2, ...).  Every wave waits until its coherent
// stores have completed (the release half: on this hardware a store counted
// complete has reached the device-coherent level), then thread 0 bumps the
// group counter; the group's last arrival bumps the release counter.  The
// wait ends when all groups are complete (or on abort / timeout); the
// coherent loads issued after it (the acquire half) see every store made
// before any arrival.
__device__ bool grid_barrier(unsigned* sy, unsigned epoch, long long limit, int* s_ok) {
  const int G = gridDim.x;
  const int g = blockIdx.x & 7;
  const int groups = G < 8 ? G : 8;
  const unsigned gsize = (unsigned)((G - g + 7) / 8);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned old =
        __hip_atomic_fetch_add(sync_group(sy, g), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == epoch * gsize - 1u)
      __hip_atomic_fetch_add(sync_release(sy), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return wait_until(sync_release(sy), epoch * (unsigned)groups, limit, s_ok);
}

// Tile steps (float4 per lane) kept in VGPRs; the rest of the tile lives in
// LDS.  At BM = 256 the whole tile takes 64 of a lane's 128 VGPRs; with 14 of
// the 16 steps in registers and 2 in LDS (32 KB per workgroup) a pass at
// n = 4000 takes 7.97 us (10 steps: 8.13 us, 12: 8.00, all 16: 8.02), measured
// on MI355X with nothing spilled.
template <int BM>
struct TileSplit {
  static constexpr int IN_REGS = BM == 256 ? SDSN_ONCHIP_REG_STEPS : TileShape<BM>::STEPS;
  static constexpr int IN_LDS = TileShape<BM>::STEPS - IN_REGS;
};

// Element stp of a lane's tile: a register or its LDS slot.
template <int BM>
struct TileStore {
  float4 r[TileSplit<BM>::IN_REGS > 0 ? TileSplit<BM>::IN_REGS : 1];
  float4 (*l)[4 * BM];
  __device__ __forceinline__ float4 get(int stp) const {
    return stp < TileSplit<BM>::IN_REGS ? r[stp] : l[stp - TileSplit<BM>::IN_REGS][threadIdx.x];
  }
  __device__ __forceinline__ void set(int stp, const float4& v) {
    if (stp < TileSplit<BM>::IN_REGS)
      r[stp] = v;
    else
      l[stp - TileSplit<BM>::IN_REGS][threadIdx.x] = v;
  }
};

template <int BM>
__global__ __launch_bounds__(4 * BM) void sdsn_onchip_kernel(OnchipArgs a) {
  using TS = TileShape<BM>;
  constexpr int NT = TS::NT;
  constexpr int LPR = TS::LPR;
  constexpr int RPW = TS::RPW;
  constexpr int STEPS = TS::STEPS;
  constexpr int IN_LDS = TileSplit<BM>::IN_LDS;
  __shared__ float4 s_tile[IN_LDS > 0 ? IN_LDS : 1][NT];
  __shared__ double s_rowsum[BM];
  __shared__ float s_colred[16][BM];
  __shared__ float s_a[BM];
  __shared__ float s_b[BM];
  __shared__ double s_red[NT / 64];
  __shared__ double s_chain[2][4][BM];
  __shared__ int s_ok;

  const int tid = threadIdx.x;
  const int G = gridDim.x;

  // ---- roll call: nothing is read or written before the whole grid is in
  if (tid == 0)
    __hip_atomic_fetch_add(sync_roll(a.sync), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!wait_until(sync_roll(a.sync), (unsigned)G, a.roll_ticks, &s_ok)) {
    if (tid == 0) atomicOr(&a.st->invalid, kInvalidRollCall);
    return;
  }

  const int lane = tid & 63;
  // Wave index as a scalar: row bounds then stay in SGPRs.
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = a.n, np = a.np, nb = np / BM;
  int t = blockIdx.x;  // tile index
  if ((G & 7) == 0) t = (t & 7) * (G >> 3) + (t >> 3);  // tile rows share an XCD
  const int bm = t / nb, bn = t % nb;
  const int q = lane / LPR;
  const int cl = (lane % LPR) * 4;
  const int j = bn * BM + cl;
  const bool c0 = j < n, c1 = j + 1 < n, c2 = j + 2 < n, c3 = j + 3 < n;

  // ---- load the tile (rows >= n and columns >= n read as zero) and emit the
  // partials and maximum of the input
  TileStore<BM> xv;
  xv.l = s_tile;
  float lmax = -INFINITY;
  float4 cacc = make_float4(0.f, 0.f, 0.f, 0.f);
  RowSums<BM> rows;
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
    xv.set(stp, v);
    tile_step_sums<BM>(v, stp, rows, cacc);
  }
  rows.finish(w, s_rowsum);
  tile_partials<BM>(cacc, s_rowsum, s_colred, s_red, a.p[0].rowp, a.p[0].colp, a.p[0].tot, bm,
                    bn, nb, np, CoherentStore());
  {
    const float tm = block_max<NT>(lmax, reinterpret_cast<float*>(s_red));
    if (tid == 0) CoherentStore()(&a.p[0].tmax[bm * nb + bn], tm);
  }

  unsigned epoch = 1;
  int k = 1;
  double gamma = 0.0;
  bool ok = true;
  const double dn = (double)n;
  // Launch constants of the P1 correction, held in scalar registers.
  const double half0 = uniform_f64(0.5 / dn), dn2 = uniform_f64(dn * dn);
  for (;; ++k, ++epoch) {
    ok = grid_barrier(a.sync, epoch, a.wait_ticks, &s_ok);
    if (!ok) break;
    const Partials in = a.p[(k - 1) & 1];
    const Partials out = a.p[k & 1];
    // The thread index as seen by this pass.  At BM = 256 an opaque copy, so
    // that the LDS addresses formed from it are formed again in every pass
    // rather than held in registers across it: at four waves per SIMD a lane
    // has 128 registers, and addresses held across the pass were spilled to
    // scratch and reloaded, each reload a full memory wait, every pass
    // (measured at n = 4000: 8.32 -> 8.13 us per pass, and with the registers
    // freed 14 tile steps instead of 10 fit in them: 7.97 us).  The smaller
    // tiles do not spill and run slightly faster without the copy.
    int tk = tid;
    if constexpr (BM == 256) asm volatile("" : "+v"(tk));
    // All reads of the previous pass's partials are issued before they are
    // combined: the tile totals, then thread (p, r)'s chains p of row r's and
    // column r's partial sums (combined in a fixed order below).  Addresses
    // are a uniform base (this tile's rows or columns) plus a per-lane offset
    // formed from the thread index, so nothing of them stays live across the
    // pass.
    double part = 0.0;
    float m = -INFINITY;
    {
      const int r = tk % BM, p = tk / BM;
      const double* rb = in.rowp + bm * BM;
      const double* cb = in.colp + bn * BM;
      auto ldr = [&](int b) { return ld_coherent(&at_u32(rb, (unsigned)(b * np + r))); };
      auto ldc = [&](int b) { return ld_coherent(&at_u32(cb, (unsigned)(b * np + r))); };
      double rsum, csum;
      if (nb <= 16) {
        // nb * nb <= NT: one total (and, on the first pass, one tile maximum)
        // per thread, read together with both chains.
        const bool has_t = tk < nb * nb;
        const unsigned tt = has_t ? (unsigned)tk : 0u;
        const double tv = ld_coherent(&at_u32(in.tot, tt));
        const float mv = (k == 1) ? ld_coherent(&at_u32(in.tmax, tt)) : -INFINITY;
        chain_sum_pair16(ldr, ldc, nb, p, rsum, csum);
        part = has_t ? part + tv : part;
        m = has_t ? fmaxf(m, mv) : m;
      } else {
#pragma unroll 1
        for (int u = tid; u < nb * nb; u += NT) part += ld_coherent(&at_u32(in.tot, (unsigned)u));
        if (k == 1)
          for (int u = tid; u < nb * nb; u += NT)
            m = fmaxf(m, ld_coherent(&at_u32(in.tmax, (unsigned)u)));
        rsum = chain_sum(ldr, nb, p);
        csum = chain_sum(ldc, nb, p);
      }
      s_chain[0][p][r] = rsum;
      s_chain[1][p][r] = csum;
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
    const double half = half0 + 0.5 * sd * S / dn2;
    if (tk < BM) {
      const double ri = combine4(s_chain[0][0][tk], s_chain[0][1][tk], s_chain[0][2][tk],
                                 s_chain[0][3][tk]);
      const double cj = combine4(s_chain[1][0][tk], s_chain[1][1][tk], s_chain[1][2][tk],
                                 s_chain[1][3][tk]);
      // Rows and columns past n get -inf, so their entries (zero) map to
      // max(0, -inf) = 0 without a test per entry.
      s_a[tk] = (bm * BM + tk < n) ? (float)(half - sd * ri / dn) : -INFINITY;
      s_b[tk] = (bn * BM + tk < n) ? (float)(half - sd * cj / dn) : -INFINITY;
    }
    __syncthreads();
    const int clk = ((tk & 63) % LPR) * 4;
    const float4 bt = make_float4(s_b[clk], s_b[clk + 1], s_b[clk + 2], s_b[clk + 3]);
    cacc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int stp = 0; stp < STEPS; ++stp) {
      const int rl = w * 16 + stp * RPW + q;
      const float ai = s_a[rl];
      const float4 x = xv.get(stp);
      float4 y;
      y.x = fmaxf(0.0f, fmaf(s, x.x, ai + bt.x));
      y.y = fmaxf(0.0f, fmaf(s, x.y, ai + bt.y));
      y.z = fmaxf(0.0f, fmaf(s, x.z, ai + bt.z));
      y.w = fmaxf(0.0f, fmaf(s, x.w, ai + bt.w));
      xv.set(stp, y);
      tile_step_sums<BM>(y, stp, rows, cacc);
    }
    rows.finish(w, s_rowsum);
    tile_partials<BM>(cacc, s_rowsum, s_colred, s_red, out.rowp, out.colp, out.tot, bm, bn, nb,
                      np, CoherentStore(), tk);
  }
  if (!ok) {
    if (tid == 0) atomicOr(&a.st->invalid, kInvalidBarrier);
    return;
  }
  const int passes = k - 1;

  if (a.dst != nullptr) {
#pragma unroll
    for (int stp = 0; stp < STEPS; ++stp) {
      const int i = bm * BM + w * 16 + stp * RPW + q;
      if (i < n) *reinterpret_cast<float4*>(&at_u32(a.dst, (unsigned)(i * np + j))) = xv.get(stp);
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
      const float4 d = xv.get(stp);
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
int resident_per_cu() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(&sdsn_onchip_kernel<BM>), 4 * BM, 0) !=
      hipSuccess)
    return 0;
  return per_cu;
}

}  // namespace

int sdsn_onchip_per_cu(int bm) {
  // Queried once per variant (the answer depends only on the kernel).
  static const int k64 = resident_per_cu<64>();
  static const int k128 = resident_per_cu<128>();
  static const int k256 = resident_per_cu<256>();
  switch (bm) {
    case 64:
      return k64;
    case 128:
      return k128;
    case 256:
      return k256;
  }
  return 0;
}

bool sdsn_onchip_fits(int device, int bm, int np) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return false;
  const long nb = np / bm;
  const int per_cu = sdsn_onchip_per_cu(bm);
  return nb * nb <= (long)per_cu * cus && nb * nb <= kOnchipMaxGrid;
}

hipError_t launch_sdsn_onchip(int bm, const OnchipArgs& a, hipStream_t s) {
  if (a.np % bm != 0 || a.n > a.np || a.n < 1 || a.sync == nullptr) return hipErrorInvalidValue;
  const int nb = a.np / bm;
  if ((long)nb * nb > kOnchipMaxGrid) return hipErrorInvalidValue;
  switch (bm) {
    case 64:
      sdsn_onchip_kernel<64><<<nb * nb, 256, 0, s>>>(a);
      break;
    case 128:
      sdsn_onchip_kernel<128><<<nb * nb, 512, 0, s>>>(a);
      break;
    case 256:
      sdsn_onchip_kernel<256><<<nb * nb, 1024, 0, s>>>(a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fram
