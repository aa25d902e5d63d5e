// Host runtime of libfram: context, workspace plan, argument validation and
// the loop driver of Algorithm 1 (outer fixed-point loop) around the device
// kernels.  Implements the C ABI declared in include/fram.h.
//
// Loop driver.  Per outer iteration the device runs GEMM 1, GEMM 2, the tile
// statistics of X, then SDSN passes.  SDSN is data-dependent (it stops when
// gamma <= gamma_tol, Sec. 5.2), so passes are enqueued in chunks: every pass
// kernel re-checks gamma of its input on the device and turns into a no-op
// once the projection is done, and the host reads the done flag once per
// chunk.  The first chunk of an iteration is sized from the previous
// iteration's pass count (which settles quickly as N converges), so in steady
// state one host synchronisation per outer iteration suffices.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <atomic>
#include <chrono>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fram.h"
#include "fram_internal.h"

using fram::DevState;
using fram::Elem;
using fram::Partials;

struct fram_ctx {
  int device = 0;
  size_t budget = 0;
  bool inited = false;
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  DevState* hst = nullptr;  // pinned host mirror of the device state
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // profiling pair
  std::string err;
  fram_stats last{};
  int fit_bm = 0, fit_np = 0, fit_ok = 0;  // cached on-chip SDSN feasibility
  unsigned* sync = nullptr;                // on-chip SDSN barrier block (own allocation)
  long long clock_khz = 0;                 // device wall-clock rate (on-chip wait bounds)
  // Asynchronous launch timing (profile = 2): event pairs recorded around
  // launches and read once the stream has passed them.
  struct Timing {
    hipEvent_t a, b;
    double* acc;
  };
  std::vector<hipEvent_t> evpool;
  size_t evused = 0;
  std::vector<Timing> pending;
  // Argmax-stability stop: the row argmax of N of this and of the previous
  // outer iteration (host copies).
  std::vector<int32_t> arg_cur, arg_prev;
  // fram_solve_many: worker contexts (own stream and workspace each), made on
  // first use and kept until fram_destroy, and the context of the lockstep
  // group of small pairs.
  std::vector<fram_ctx*> workers;
  fram_ctx* group = nullptr;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Tile table set by fram_set_tile_table (an autotuner's choice per size
// bucket), shared by every context of the process: bucket k covers
// n_max[k-1] < n <= n_max[k].
constexpr int kMaxTileBuckets = 64;
std::mutex g_tile_mu;
int g_tile_count = 0;
int g_tile_nmax[kMaxTileBuckets];
int g_tile_edge[kMaxTileBuckets];

int choose_tile(int n, int requested) {
  if (requested == 64 || requested == 128 || requested == 256) return requested;
  {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    for (int k = 0; k < g_tile_count; ++k)
      if (n <= g_tile_nmax[k]) return g_tile_edge[k];
  }
  // Up to 128 the matrix is one tile and a projection is one launch.
  if (n <= 64) return 64;
  if (n <= 128) return 128;
  const int cands[3] = {256, 128, 64};
  for (int bm : cands) {
    const long nb = (n + bm - 1) / bm;
    if (nb * nb >= 200) return bm;
  }
  return 64;
}

struct Layout {
  int bm = 64, np = 64, nb = 1;
  Elem e = Elem::F32;
  size_t A64 = 0, B64 = 0, K64 = 0, Kp = 0, Alp = 0, Blp = 0, W = 0, N = 0, Nlp = 0, X = 0;
  size_t Nprev = 0;  // DSPFP: the iterate before the update
  size_t rowp[2] = {0, 0}, colp[2] = {0, 0}, tot[2] = {0, 0}, tmax[2] = {0, 0};
  size_t upd = 0, mx = 0, obj = 0, sigma = 0, lap = 0, state = 0;
  int nupd = 1, nmax = 1, nobj = 1;
  size_t total = 0;
};

enum class Use { Solve, SolveDev, Sdsn, Gradient };

Layout plan(int n, Elem e, int tile, Use use, bool node = false, bool dspfp = false) {
  Layout L;
  L.e = e;
  L.bm = choose_tile(n, tile);
  L.np = (n + L.bm - 1) / L.bm * L.bm;
  L.nb = L.np / L.bm;
  const size_t np2 = (size_t)L.np * L.np;
  const size_t es = fram::elem_size(e);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align_up(bytes);
    return at;
  };
  if (use == Use::Solve) {
    L.A64 = take((size_t)n * n * 8);
    L.B64 = take((size_t)n * n * 8);
    if (node) L.K64 = take((size_t)n * n * 8);
  }
  if (node) L.Kp = take(np2 * 4);
  const bool gemm = use != Use::Sdsn;
  if (gemm) {
    L.Alp = take(np2 * es);
    L.Blp = take(np2 * es);
    L.W = take(np2 * es);
    L.Nlp = (e == Elem::F32) ? 0 : take(np2 * es);
  }
  L.X = take(np2 * 4);
  if (use == Use::Solve || use == Use::SolveDev || use == Use::Gradient) L.N = take(np2 * 4);
  if (dspfp) L.Nprev = take(np2 * 4);
  for (int k = 0; k < 2; ++k) {
    L.rowp[k] = take((size_t)L.nb * L.np * 8);
    L.colp[k] = take((size_t)L.nb * L.np * 8);
    L.tot[k] = take((size_t)L.nb * L.nb * 8);
    L.tmax[k] = take((size_t)L.nb * L.nb * 4);
  }
  L.nupd = fram::update_blocks(n);
  L.nmax = fram::max_blocks(n);
  L.nobj = fram::objective_blocks(n);
  L.upd = take((size_t)std::max(L.nupd, L.nb * L.nb) * 16);
  L.mx = take((size_t)L.nmax * 16);
  L.obj = take((size_t)L.nobj * 8);
  L.sigma = take((size_t)n * 4);
  if (use == Use::Solve || use == Use::SolveDev) L.lap = take(fram::lap_workspace_bytes(n));
  L.state = take(sizeof(DevState));
  L.total = off;
  return L;
}

bool valid_prec(int p) { return p == FRAM_FP32 || p == FRAM_BF16 || p == FRAM_FP16; }

// Devices whose on-chip SDSN launches are ordered (see OnchipGate).
constexpr int kMaxGateDevices = 64;
// Most worker contexts of one fram_solve_many call (fram_options.many_workers).
constexpr int kMaxManyWorkers = 32;
// Largest accepted on-chip wait bound (fram_options.onchip_*_us): one minute.
constexpr int kMaxOnchipWaitUs = 60000000;

fram_status check_options(const fram_options& o) {
  if (!valid_prec((int)o.prec)) return FRAM_EINVAL;
  if (!(o.alpha > 0.0 && o.alpha <= 1.0)) return FRAM_EINVAL;
  if (!(o.gamma_tol >= 0.0) || !std::isfinite(o.gamma_tol)) return FRAM_EINVAL;
  if (o.sdsn_max < 1) return FRAM_EINVAL;
  if (!(o.tile == 0 || o.tile == 64 || o.tile == 128 || o.tile == 256)) return FRAM_EINVAL;
  if (o.profile < 0 || o.profile > 2) return FRAM_EINVAL;
  if (o.sdsn_mode < 0 || o.sdsn_mode > 2) return FRAM_EINVAL;
  if (o.stable_iters < 0) return FRAM_EINVAL;
  if (o.stall_iters < 0 || !(o.stall_delta > 0.0) || !std::isfinite(o.stall_delta))
    return FRAM_EINVAL;
  if (o.variant != 0 && o.variant != 1) return FRAM_EINVAL;
  if (o.dsn_iters < 1) return FRAM_EINVAL;
  if (o.many_workers < 1 || o.many_workers > kMaxManyWorkers) return FRAM_EINVAL;
  if (o.onchip_roll_us < 0 || o.onchip_roll_us > kMaxOnchipWaitUs) return FRAM_EINVAL;
  if (o.onchip_barrier_us < 0 || o.onchip_barrier_us > kMaxOnchipWaitUs) return FRAM_EINVAL;
  return FRAM_OK;
}

fram_status check_scalars(int n, double theta, int iters, double tol) {
  if (n < 1 || n > FRAM_MAX_N) return FRAM_EINVAL;
  if (!(theta > 0.0) || !std::isfinite(theta)) return FRAM_EINVAL;
  if (iters < 1) return FRAM_EINVAL;
  if (!(tol >= 0.0) || !std::isfinite(tol)) return FRAM_EINVAL;
  return FRAM_OK;
}

// A host warm start must be finite.
fram_status check_warm(const fram_options& o, int n) {
  if (o.N0 == nullptr) return FRAM_OK;
  for (size_t t = 0; t < (size_t)n * n; ++t)
    if (!std::isfinite(o.N0[t])) return FRAM_EINVAL;
  return FRAM_OK;
}

// Sec. 3: A is nonnegative and symmetric; entries must also be finite.
fram_status check_graph(const double* A, int n) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double v = A[(size_t)i * n + j];
      if (!std::isfinite(v) || v < 0.0) return FRAM_EINVAL;
      if (j > i && A[(size_t)j * n + i] != v) return FRAM_EINVAL;
    }
  return FRAM_OK;
}

#define HIPCHK(call)                                                   \
  do {                                                                 \
    hipError_t e_ = (call);                                            \
    if (e_ != hipSuccess) {                                            \
      c->err = std::string(#call) + ": " + hipGetErrorString(e_);      \
      return FRAM_EDEVICE;                                             \
    }                                                                  \
  } while (0)

fram_status ensure_device(fram_ctx* c) {
  HIPCHK(hipSetDevice(c->device));
  if (c->inited) return FRAM_OK;
  HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  HIPCHK(hipHostMalloc((void**)&c->hst, sizeof(DevState), hipHostMallocDefault));
  HIPCHK(hipEventCreate(&c->ev0));
  HIPCHK(hipEventCreate(&c->ev1));
  // Barrier counters of the on-chip SDSN launches (zeroed before each launch).
  HIPCHK(hipMalloc((void**)&c->sync, fram::kOnchipSyncBytes));
  int khz = 0;
  HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device));
  c->clock_khz = khz > 0 ? khz : 100000;
  c->inited = true;
  return FRAM_OK;
}

fram_status ensure_ws(fram_ctx* c, size_t bytes) {
  if (c->budget != 0 && bytes > c->budget) {
    c->err = "workspace exceeds the HBM budget";
    return FRAM_ENOMEM;
  }
  if (c->ws_bytes >= bytes) return FRAM_OK;
  if (c->ws) {
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  hipError_t e = hipMalloc(&c->ws, bytes);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    c->err = "device allocation failed";
    return FRAM_ENOMEM;
  }
  HIPCHK(e);
  c->ws_bytes = bytes;
  return FRAM_OK;
}

template <typename T>
T* at(fram_ctx* c, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(c->ws) + off);
}

Partials partials(fram_ctx* c, const Layout& L, int k) {
  Partials p;
  p.rowp = at<double>(c, L.rowp[k]);
  p.colp = at<double>(c, L.colp[k]);
  p.tot = at<double>(c, L.tot[k]);
  p.tmax = at<float>(c, L.tmax[k]);
  return p;
}

fram_status read_state(fram_ctx* c, DevState* dst, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(c->hst, dst, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return FRAM_OK;
}

// Profiling.  mode 1: each timed launch is bracketed by two events on its
// stream and waited for, so the elapsed time is that launch alone (launches
// serialised).  mode 2: the events are only recorded; their times are
// collected by flush_timings once the stream has passed them, so the launches
// keep their normal overlap and host pacing.
struct Prof {
  int mode = 0;
  fram_ctx* c = nullptr;
  hipStream_t s = nullptr;
  float last_ms = 0.0f;
};

fram_status take_events(fram_ctx* c, hipEvent_t* a, hipEvent_t* b) {
  while (c->evpool.size() < c->evused + 2) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->evpool.push_back(e);
  }
  *a = c->evpool[c->evused++];
  *b = c->evpool[c->evused++];
  return FRAM_OK;
}

// Adds the elapsed time of every pending event pair to its counter.
fram_status flush_timings(fram_ctx* c) {
  for (const auto& t : c->pending) {
    HIPCHK(hipEventSynchronize(t.b));
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, t.a, t.b));
    if (t.acc) *t.acc += ms;
  }
  c->pending.clear();
  c->evused = 0;
  return FRAM_OK;
}

template <typename F>
fram_status timed(Prof& p, double* acc, int* cnt, F&& launch) {
  fram_ctx* c = p.c;
  if (p.mode == 0) {
    HIPCHK(launch());
    return FRAM_OK;
  }
  if (p.mode == 2) {
    hipEvent_t a, b;
    fram_status r = take_events(c, &a, &b);
    if (r != FRAM_OK) return r;
    HIPCHK(hipEventRecord(a, p.s));
    HIPCHK(launch());
    HIPCHK(hipEventRecord(b, p.s));
    c->pending.push_back({a, b, acc});
    if (cnt) *cnt += 1;
    return FRAM_OK;
  }
  HIPCHK(hipEventRecord(c->ev0, p.s));
  HIPCHK(launch());
  HIPCHK(hipEventRecord(c->ev1, p.s));
  HIPCHK(hipEventSynchronize(c->ev1));
  HIPCHK(hipEventElapsedTime(&p.last_ms, c->ev0, c->ev1));
  if (acc) *acc += p.last_ms;
  if (cnt) *cnt += 1;
  return FRAM_OK;
}

// Runs SDSN passes on X (already holding the input, partial set 0 filled by
// the tile statistics).  Returns passes made in *passes.
fram_status run_sdsn_passes(fram_ctx* c, const Layout& L, int n, float* X, DevState* st,
                            double theta, const fram_options& o, int first_chunk,
                            hipStream_t s, int* passes, double* gamma, bool* capped,
                            fram_stats* stt, double fixed_scale = 0.0) {
  int k = 1;
  const int last = o.sdsn_max + 1;  // pass index that only evaluates gamma
  int chunk = std::max(2, first_chunk);
  if (o.profile == 1) {
    // One pass at a time; the launch that only finds gamma <= gamma_tol is
    // not counted as a pass.
    Prof p{1, c, s, 0.0f};
    for (int kk = 1; kk <= last; ++kk) {
      fram_status r = timed(p, nullptr, nullptr, [&] {
        return fram::launch_sdsn_pass(L.bm, X, n, L.np, partials(c, L, (kk - 1) & 1),
                                      partials(c, L, kk & 1), st, kk, o.sdsn_max, theta,
                                      o.gamma_tol, s, fixed_scale);
      });
      if (r != FRAM_OK) return r;
      r = read_state(c, st, s);
      if (r != FRAM_OK) return r;
      if (c->hst->done) break;
      stt->ms_sdsn += p.last_ms;
      stt->sdsn_launches += 1;
    }
    k = last + 1;
  }
  if (L.nb == 1 && o.profile != 1) {
    // A single tile: the whole projection is one workgroup launch.
    Prof p{o.profile, c, s, 0.0f};
    fram_status r0 = timed(p, &stt->ms_sdsn, nullptr, [&] {
      return fram::launch_sdsn_chunk(L.bm, X, n, L.np, partials(c, L, 0), partials(c, L, 1), st,
                                     1, last, o.sdsn_max, theta, o.gamma_tol, s, fixed_scale);
    });
    if (r0 != FRAM_OK) return r0;
    fram_status r = read_state(c, st, s);
    if (r != FRAM_OK) return r;
    if (!c->hst->done) {
      c->err = "SDSN loop ended without completion flag";
      return FRAM_EDEVICE;
    }
  }
  while (o.profile != 1 && L.nb != 1) {
    const int end = std::min(last, k + chunk - 1);
    Prof p{o.profile, c, s, 0.0f};
    fram_status r0 = timed(p, &stt->ms_sdsn, nullptr, [&] {
      for (int kk = k; kk <= end; ++kk) {
        const hipError_t e = fram::launch_sdsn_pass(L.bm, X, n, L.np, partials(c, L, (kk - 1) & 1),
                                                    partials(c, L, kk & 1), st, kk, o.sdsn_max,
                                                    theta, o.gamma_tol, s, fixed_scale);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    });
    if (r0 != FRAM_OK) return r0;
    k = end + 1;
    fram_status r = read_state(c, st, s);
    if (r != FRAM_OK) return r;
    if (c->hst->done) break;
    if (k > last) {
      c->err = "SDSN loop ended without completion flag";
      return FRAM_EDEVICE;
    }
    chunk = 4;
  }
  *passes = c->hst->passes;
  *gamma = c->hst->gamma;
  *capped = (*passes >= o.sdsn_max) && !(*gamma <= o.gamma_tol);
  if (!std::isfinite(*gamma)) {
    c->err = "non-finite gamma in SDSN";
    return FRAM_ENUMERIC;
  }
  return FRAM_OK;
}

// Decide whether the on-chip SDSN path is used for this layout.
// Automatic mode takes the on-chip launch whenever the grid fits the device
// (and a single-tile matrix, whose streaming projection is already one
// workgroup launch, streams); "stream" never does; "onchip" insists.
fram_status use_onchip(fram_ctx* c, const Layout& L, const fram_options& o, bool* on) {
  *on = false;
  if (o.sdsn_mode == 1) return FRAM_OK;
  const bool insist = o.sdsn_mode == 2;
  if (!insist && L.nb == 1) return FRAM_OK;
  // Barrier counters reach (passes + 2) * ceil(grid / 8) < 2^32.
  if (o.sdsn_max > (1 << 22) || c->device >= kMaxGateDevices) {
    if (!insist) return FRAM_OK;
    c->err = "sdsn_max too large or device index too high for the on-chip SDSN path";
    return FRAM_EINVAL;
  }
  if (c->fit_bm != L.bm || c->fit_np != L.np) {
    c->fit_bm = L.bm;
    c->fit_np = L.np;
    c->fit_ok = fram::sdsn_onchip_fits(c->device, L.bm, L.np) ? 1 : 0;
  }
  if (!c->fit_ok) {
    if (!insist) return FRAM_OK;
    c->err = "on-chip SDSN does not fit this device";
    return FRAM_EINVAL;
  }
  *on = true;
  return FRAM_OK;
}

// Default bounds on the waits of the on-chip SDSN (fram_options.onchip_*_us
// override them).  The roll call (all workgroups resident) normally completes
// within microseconds; when kernels of other streams hold compute units
// longer than this, the launch is abandoned and the projection streams
// instead.  A pass barrier takes a few microseconds; a wait thousands of
// times longer means a workgroup has stopped running (its hardware queue was
// preempted, which happens when a process's queues outnumber those the
// device schedules at once), and the grid gives up, writes nothing and the
// projection streams: holding the other compute units until the queue
// returns would only stall everything else.
constexpr long long kRollCallUs = 10000;
constexpr long long kBarrierUs = 20000;

// Compute-unit budget of the on-chip SDSN launches of the process on a device.
// A grid of G workgroups of which `per_cu` fit on one compute unit occupies
// G / per_cu compute units.  Before a launch, the launches that may still be
// running are counted; while they and the new grid together would need more
// compute units than the device has, the new launch waits (on the device, for
// the completion event) for the oldest of them.  So the grids that can run at
// the same time always fit on the device together: many small projections
// (small pairs solved concurrently) overlap, and a grid that needs the whole
// device (n = 4000) runs alone.  Every wait points back to an earlier launch,
// so the waits cannot form a cycle.  The roll call in the kernel still guards
// against compute units held by other kernels.
struct OnchipGate {
  std::mutex mu;
  struct Live {
    hipEvent_t ev;
    double cus;
  };
  std::deque<Live> live;         // launches that may still run, oldest first
  std::vector<hipEvent_t> idle;  // events of completed launches, for reuse
  int cus = 0;                   // compute units of the device
};
OnchipGate g_gate[kMaxGateDevices];

// One on-chip projection: D = SDSN(src) with every pass in one launch;
// optionally writes D to dst (ld np) and/or applies the N update.  Whether it
// ran (or the roll call failed and nothing was done) is in st->invalid.
fram_status run_sdsn_onchip(fram_ctx* c, const Layout& L, int n, const float* src, int ld_src,
                            float* dst, float* N, void* Nlp, Elem e, double alpha,
                            DevState* st, double theta, const fram_options& o, hipStream_t s) {
  fram::OnchipArgs a{};
  a.src = src;
  a.ld_src = ld_src;
  a.src_vec = (ld_src % 4 == 0 && (reinterpret_cast<uintptr_t>(src) % 16) == 0) ? 1 : 0;
  a.dst = dst;
  a.n = n;
  a.np = L.np;
  a.p[0] = partials(c, L, 0);
  a.p[1] = partials(c, L, 1);
  a.st = st;
  a.sync = c->sync;
  a.roll_ticks = c->clock_khz * (o.onchip_roll_us > 0 ? o.onchip_roll_us : kRollCallUs) / 1000;
  a.wait_ticks =
      c->clock_khz * (o.onchip_barrier_us > 0 ? o.onchip_barrier_us : kBarrierUs) / 1000;
  a.max_passes = o.sdsn_max;
  a.theta = theta;
  a.gamma_tol = o.gamma_tol;
  a.N = N;
  a.Nlp = (e == Elem::F32) ? nullptr : Nlp;
  a.nlp_kind = (N == nullptr || e == Elem::F32) ? 0 : (e == Elem::BF16 ? 1 : 2);
  a.alpha = (float)alpha;
  a.dpart = at<double>(c, L.upd);
  OnchipGate& g = g_gate[c->device];
  std::lock_guard<std::mutex> lk(g.mu);
  if (g.cus == 0) HIPCHK(hipDeviceGetAttribute(&g.cus, hipDeviceAttributeMultiprocessorCount,
                                               c->device));
  const int per_cu = std::max(1, fram::sdsn_onchip_per_cu(L.bm));
  const double need = std::min((double)g.cus, (double)L.nb * L.nb / per_cu);
  // Forget launches that have completed.
  double used = 0.0;
  for (auto it = g.live.begin(); it != g.live.end();) {
    const hipError_t q = hipEventQuery(it->ev);
    if (q == hipSuccess) {
      g.idle.push_back(it->ev);
      it = g.live.erase(it);
    } else {
      if (q != hipErrorNotReady) HIPCHK(q);
      used += it->cus;
      ++it;
    }
  }
  // Wait for the oldest launches until this grid fits beside the rest.
  while (!g.live.empty() && used + need > (double)g.cus + 1e-9) {
    HIPCHK(hipStreamWaitEvent(s, g.live.front().ev, 0));
    used -= g.live.front().cus;
    g.live.pop_front();  // this launch starts after it: no longer counted
  }
  hipEvent_t ev = nullptr;
  if (!g.idle.empty()) {
    ev = g.idle.back();
    g.idle.pop_back();
  } else {
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
  HIPCHK(fram::launch_zero(c->sync, fram::kOnchipSyncBytes, s));
  HIPCHK(fram::launch_sdsn_onchip(L.bm, a, s));
  HIPCHK(hipEventRecord(ev, s));
  g.live.push_back({ev, need});
  return FRAM_OK;
}

bool is_permutation(const int32_t* p, int n) {
  std::vector<char> seen(n, 0);
  for (int i = 0; i < n; ++i) {
    const int j = p[i];
    if (j < 0 || j >= n || seen[j]) return false;
    seen[j] = 1;
  }
  return true;
}

// Optional node term of eq. (1) / eq. (3): X gains w K (K n x n FP64, device).
struct NodeTerm {
  const double* K = nullptr;
  double w = 0.0;
};

fram_status finish_discretise(fram_ctx* c, const Layout& L, int n, const double* dA,
                              const double* dB, const NodeTerm& nt, float* N, int32_t* dsig,
                              DevState* st, hipStream_t s, int32_t* perm, double* obj,
                              int* lap_paths, Prof& prof, fram_stats* stt) {
  // Row argmax of N with the starting duals, then the exact assignment on the
  // device (nothing to augment when the argmax is a permutation).
  char* lws = at<char>(c, L.lap);
  double* u = reinterpret_cast<double*>(lws);
  fram_status q = timed(prof, &stt->ms_discretize, nullptr, [&] {
    hipError_t e = fram::launch_row_argmax(N, n, L.np, dsig, s, u);
    if (e != hipSuccess) return e;
    fram::LapProblem lp{N, n, L.np, dsig, lws, u, 1, &st->lap_paths};
    return fram::launch_lap(&lp, nullptr, 1, n, s);
  });
  if (q != FRAM_OK) return q;
  HIPCHK(fram::launch_objective(dA, dB, dsig, n, at<double>(c, L.obj), L.nobj, st, s));
  if (nt.K != nullptr) HIPCHK(fram::launch_node_objective(nt.K, dsig, n, nt.w, st, s));
  HIPCHK(hipMemcpyAsync(perm, dsig, (size_t)n * 4, hipMemcpyDeviceToHost, s));
  fram_status r = read_state(c, st, s);
  if (r != FRAM_OK) return r;
  *lap_paths = c->hst->lap_paths;
  if (!is_permutation(perm, n)) {
    c->err = "the assignment of N failed (non-finite entries)";
    return FRAM_ENUMERIC;
  }
  *obj = c->hst->objective;
  if (!std::isfinite(*obj)) {
    c->err = "non-finite objective";
    return FRAM_ENUMERIC;
  }
  return FRAM_OK;
}

// Algorithm 1 on device inputs dA, dB (n x n FP64, ld n).
fram_status run_solve(fram_ctx* c, const Layout& L, const double* dA, const double* dB,
                      const NodeTerm& nt, int n, double theta, int iters, double tol,
                      const fram_options& o, bool validate_dev, hipStream_t s, int32_t* perm,
                      double* obj, fram_stats* stt) {
  const Elem e = L.e;
  const size_t np2 = (size_t)L.np * L.np;
  DevState* st = at<DevState>(c, L.state);
  void* Alp = at<void>(c, L.Alp);
  void* Blp = at<void>(c, L.Blp);
  void* W = at<void>(c, L.W);
  float* N = at<float>(c, L.N);
  void* Nlp = (e == Elem::F32) ? (void*)N : at<void>(c, L.Nlp);
  float* X = at<float>(c, L.X);
  int32_t* dsig = at<int32_t>(c, L.sigma);

  c->pending.clear();
  c->evused = 0;
  HIPCHK(fram::launch_zero(st, sizeof(DevState), s));
  if (validate_dev) {
    if (nt.K != nullptr) {  // K may be signed and asymmetric; only finiteness counts
      HIPCHK(fram::launch_validate(nt.K, n, st, s));
      fram_status r = read_state(c, st, s);
      if (r != FRAM_OK) return r;
      if (c->hst->invalid & 1) {
        c->err = "device node similarities are non-finite";
        return FRAM_EINVAL;
      }
      HIPCHK(fram::launch_zero(st, sizeof(DevState), s));
    }
    HIPCHK(fram::launch_validate(dA, n, st, s));
    HIPCHK(fram::launch_validate(dB, n, st, s));
    fram_status r = read_state(c, st, s);
    if (r != FRAM_OK) return r;
    if (c->hst->invalid) {
      c->err = "device input is non-finite, negative or asymmetric";
      return FRAM_EINVAL;
    }
  }
  // Algorithm 1, steps 2-3 (each matrix scaled by its own maximum; SDSN's
  // max-normalisation makes the scale immaterial in exact arithmetic).
  HIPCHK(fram::launch_maxes(dA, dB, n, at<double>(c, L.mx), L.nmax, st, s));
  HIPCHK(fram::launch_cast_scaled(e, dA, n, Alp, L.np, st, 0, s));
  HIPCHK(fram::launch_cast_scaled(e, dB, n, Blp, L.np, st, 1, s));
  float* Kp = nullptr;
  if (nt.K != nullptr) {
    Kp = at<float>(c, L.Kp);
    HIPCHK(fram::launch_node_term(nt.K, n, nt.w, Kp, L.np, at<double>(c, L.mx), L.nmax, st, s));
  }
  // Algorithm 1, step 1: N^(0) = 0, or the caller's warm start N0 (n x n,
  // ld n, host or device memory) with zero padding.
  HIPCHK(fram::launch_zero(N, np2 * 4, s));
  if (o.N0 != nullptr) {
    HIPCHK(hipMemcpy2DAsync(N, (size_t)L.np * 4, o.N0, (size_t)n * 4, (size_t)n * 4, n,
                            hipMemcpyDefault, s));
    if (e != Elem::F32) {
      // The GEMM-type copy is cast from a contiguous copy (X is free here),
      // with the same rounding the update kernel uses.
      HIPCHK(hipMemcpyAsync(X, o.N0, (size_t)n * n * 4, hipMemcpyDefault, s));
      HIPCHK(fram::launch_cast_f32(e, X, n, Nlp, L.np, s));
    }
  } else if (e != Elem::F32) {
    HIPCHK(fram::launch_zero(Nlp, np2 * fram::elem_size(e), s));
  }

  // DSPFP variant (Sec. 4, eq. iter.DSPFP): the same outer loop, but the
  // projection is the plain alternating one on the gradient itself (first
  // pass scale maxA * maxB undoes the prescale; no theta, no division by
  // max X), with a fixed number of passes, and the outer stop is DSPFP's
  // max-abs criterion (App. B.2), reported in place of delta.
  const bool dspfp = o.variant == 1;
  fram_options os = o;
  double fixed_scale = 0.0;
  float* Nprev = nullptr;
  if (dspfp) {
    if (nt.K != nullptr) {
      c->err = "the DSPFP variant takes no node term";
      return FRAM_EINVAL;
    }
    os.gamma_tol = -2.0;  // gamma >= -1 always: never stop early
    os.sdsn_max = o.dsn_iters;
    fram_status r = read_state(c, st, s);
    if (r != FRAM_OK) return r;
    const double ma = c->hst->maxA, mb = c->hst->maxB;
    fixed_scale = (ma > 0.0 && mb > 0.0) ? ma * mb : 1.0;
    Nprev = at<float>(c, L.Nprev);
  }

  int total_passes = 0, last_passes = 0, max_passes_seen = 0, it = 0;
  int total_passes_streamed = 0;
  bool any_capped = false, converged = false;
  double gamma = 0.0, delta = 0.0;
  int est = 8;
  int stable = 0;
  bool prev_perm = false;
  int stall = 0;
  bool stalled = false;
  double dmin = 0.0;  // smallest delta since delta first fell to stall_delta (0: not yet)
  Prof prof{o.profile, c, s, 0.0f};
  bool onchip = false;
  if (!dspfp) {
    fram_status q = use_onchip(c, L, o, &onchip);
    if (q != FRAM_OK) return q;
  }
  for (it = 1; it <= iters; ++it) {
    // Step 5: X = A N B as W = B N^T, X = A W^T.
    fram_status r = timed(prof, &stt->ms_gemm, &stt->gemm_launches, [&] {
      return fram::launch_gemm_nt(e, L.bm, Blp, Nlp, W, false, n, L.np, L.np, s);
    });
    if (r != FRAM_OK) return r;
    r = timed(prof, &stt->ms_gemm, &stt->gemm_launches, [&] {
      return fram::launch_gemm_nt(e, L.bm, Alp, W, X, true, n, L.np, L.np, s, Kp);
    });
    if (r != FRAM_OK) return r;
    bool streamed = !onchip;
    bool state_fresh = false;  // c->hst holds the state after this iteration's update
    if (onchip) {
      // Steps 6-8 in one launch (+ the delta reduction), then the state: the
      // launch either ran every pass or, when its roll call failed, did
      // nothing, and this iteration's projection streams instead.
      r = timed(prof, &stt->ms_sdsn, nullptr, [&] {
        fram_status q = run_sdsn_onchip(c, L, n, X, L.np, nullptr, N, Nlp, e, o.alpha, st,
                                        theta, o, s);
        return q == FRAM_OK ? hipSuccess : hipErrorUnknown;
      });
      if (r != FRAM_OK) return r;
      r = timed(prof, &stt->ms_update, nullptr, [&] {
        return fram::launch_delta_final(at<double>(c, L.upd), L.nb * L.nb, st, s);
      });
      if (r != FRAM_OK) return r;
      r = read_state(c, st, s);
      if (r != FRAM_OK) return r;
      if (c->hst->invalid & (fram::kInvalidRollCall | fram::kInvalidBarrier)) {
        // The launch wrote neither X nor N: stream this iteration's
        // projection from the same X.
        HIPCHK(fram::launch_zero(&st->invalid, sizeof(int), s));
        stt->sdsn_fallbacks += 1;
        streamed = true;
      } else {
        const int passes = c->hst->passes;
        gamma = c->hst->gamma;
        if (!std::isfinite(gamma)) {
          c->err = "non-finite gamma in SDSN";
          return FRAM_ENUMERIC;
        }
        total_passes += passes;
        last_passes = passes;
        max_passes_seen = std::max(max_passes_seen, passes);
        any_capped = any_capped || (passes >= o.sdsn_max && !(gamma <= o.gamma_tol));
        stt->sdsn_onchip += 1;
        state_fresh = true;
      }
    }
    if (streamed) {
      r = timed(prof, &stt->ms_stats, nullptr, [&] {
        return fram::launch_tile_stats(L.bm, X, L.np, nullptr, n, L.np, partials(c, L, 0), st,
                                       s);
      });
      if (r != FRAM_OK) return r;
      // Step 6: D = SDSN(X, theta), in place in X.
      int passes = 0;
      bool capped = false;
      r = run_sdsn_passes(c, L, n, X, st, theta, os, est + 1, s, &passes, &gamma, &capped, stt,
                          fixed_scale);
      if (r != FRAM_OK) return r;
      est = passes;
      total_passes += passes;
      total_passes_streamed += passes;
      last_passes = passes;
      max_passes_seen = std::max(max_passes_seen, passes);
      any_capped = any_capped || capped;
      // Steps 7-8: N update and delta.
      if (dspfp) HIPCHK(fram::launch_copy_f32(N, L.np, Nprev, L.np, n, s));
      r = timed(prof, &stt->ms_update, nullptr, [&] {
        return fram::launch_update(e, X, N, Nlp, n, L.np, o.alpha, at<double>(c, L.upd),
                                   L.nupd, st, s);
      });
      if (r != FRAM_OK) return r;
      if (dspfp)
        HIPCHK(fram::launch_dspfp_criterion(N, Nprev, n, L.np, at<double>(c, L.mx), L.nmax, st,
                                            s));
    }
    // Argmax-stability stop: the row argmax of N (device) is copied back with
    // the state; the host compares it with the previous iteration's.
    const bool track = o.stable_iters > 0;
    if (track) {
      HIPCHK(fram::launch_row_argmax(N, n, L.np, dsig, s));
      c->arg_cur.resize(n);
      HIPCHK(hipMemcpyAsync(c->arg_cur.data(), dsig, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    }
    const bool watch_stall = o.stall_iters > 0;
    if (tol > 0.0 || track || watch_stall || it == iters) {
      if (!state_fresh || track) {
        r = read_state(c, st, s);
        if (r != FRAM_OK) return r;
      }
      delta = c->hst->delta;
      // DSPFP's criterion is +inf while the previous iterate is 0.
      if (dspfp ? std::isnan(delta) : !std::isfinite(delta)) {
        c->err = "non-finite delta";
        return FRAM_ENUMERIC;
      }
      if (delta <= tol) {
        converged = true;
        break;
      }
      if (watch_stall && delta <= o.stall_delta) {
        // Delta-stall rule (same as the oracle): stall_iters iterations in a
        // row without a new smallest delta since delta reached stall_delta.
        stall = (dmin > 0.0 && delta >= dmin) ? stall + 1 : 0;
        dmin = (dmin > 0.0) ? std::min(dmin, delta) : delta;
        if (stall >= o.stall_iters) {
          converged = true;
          stalled = true;
          break;
        }
      }
      if (track) {
        // Same rule as the oracle: count consecutive iterations whose argmax is
        // a permutation equal to the previous (also a permutation) one.
        const bool is_perm = is_permutation(c->arg_cur.data(), n);
        const bool same = prev_perm && c->arg_prev == c->arg_cur;
        stable = (is_perm && prev_perm && same) ? stable + 1 : 0;
        prev_perm = is_perm;
        std::swap(c->arg_prev, c->arg_cur);
        if (stable >= o.stable_iters) {
          converged = true;
          break;
        }
      }
    }
  }
  if (it > iters) it = iters;
  if (o.N_out != nullptr)
    HIPCHK(hipMemcpy2DAsync(o.N_out, (size_t)n * 4, N, (size_t)L.np * 4, (size_t)n * 4, n,
                            hipMemcpyDefault, s));
  int lap_paths = 0;
  fram_status r = finish_discretise(c, L, n, dA, dB, nt, N, dsig, st, s, perm, obj, &lap_paths,
                                    prof, stt);
  if (r != FRAM_OK) return r;
  r = flush_timings(c);
  if (r != FRAM_OK) return r;
  if (o.profile == 1) stt->sdsn_launches += stt->sdsn_onchip;  // streamed passes counted
  if (o.profile == 2) stt->sdsn_launches = total_passes_streamed + stt->sdsn_onchip;
  stt->outer_iters = it;
  stt->sdsn_passes = total_passes;
  stt->sdsn_passes_last = last_passes;
  stt->sdsn_passes_max = max_passes_seen;
  stt->converged = converged ? 1 : 0;
  stt->sdsn_capped = any_capped ? 1 : 0;
  stt->lap_paths = lap_paths;
  stt->stalled = stalled ? 1 : 0;
  stt->gemm_tile = L.bm;
  stt->delta = delta;
  stt->gamma = gamma;
  return FRAM_OK;
}

fram_options defaults() {
  fram_options o;
  fram_default_options(&o);
  return o;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

fram_status solve_host_impl(fram_ctx* c, const double* A, const double* B, const double* K,
                            double w, int n, double theta, int iters, double tol,
                            const fram_options& o, int32_t* perm, double* obj, fram_stats* stt) {
  const double t0 = now_ms();
  if (n == 1) {
    perm[0] = 0;
    *obj = A[0] * B[0] + (K ? 2.0 * w * K[0] : 0.0);
    stt->ms_total = now_ms() - t0;
    return FRAM_OK;
  }
  const Layout L = plan(n, (Elem)o.prec, o.tile, Use::Solve, K != nullptr, o.variant == 1);
  if (c->budget != 0 && L.total > c->budget) {
    c->err = "workspace exceeds the HBM budget";
    return FRAM_ENOMEM;
  }
  fram_status r = ensure_device(c);
  if (r != FRAM_OK) return r;
  r = ensure_ws(c, L.total);
  if (r != FRAM_OK) return r;
  hipStream_t s = c->stream;
  double* dA = at<double>(c, L.A64);
  double* dB = at<double>(c, L.B64);
  HIPCHK(hipMemcpyAsync(dA, A, (size_t)n * n * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dB, B, (size_t)n * n * 8, hipMemcpyHostToDevice, s));
  NodeTerm nt;
  if (K != nullptr) {
    nt.K = at<double>(c, L.K64);
    nt.w = w;
    HIPCHK(hipMemcpyAsync(at<double>(c, L.K64), K, (size_t)n * n * 8, hipMemcpyHostToDevice, s));
  }
  r = run_solve(c, L, dA, dB, nt, n, theta, iters, tol, o, false, s, perm, obj, stt);
  stt->ms_total = now_ms() - t0;
  return r;
}

// Device-input solve shared by fram_solve_dev and fram_solve_attr_dev.
fram_status solve_dev_impl(fram_ctx* c, const double* dA, const double* dB, const double* dK,
                           double w, int n, double lambda, int iters, double tol,
                           const fram_options& o, int32_t* perm_out, double* objective_out,
                           fram_stats* stats, void* stream) {
  const double t0 = now_ms();
  const Layout L = plan(n, (Elem)o.prec, o.tile, Use::SolveDev, dK != nullptr, o.variant == 1);
  if (c->budget != 0 && L.total > c->budget) {
    c->err = "workspace exceeds the HBM budget";
    return FRAM_ENOMEM;
  }
  fram_status r = ensure_device(c);
  if (r != FRAM_OK) return r;
  r = ensure_ws(c, L.total);
  if (r != FRAM_OK) return r;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  fram_stats st{};
  if (n == 1) {
    double a = 0, b = 0, k = 0;
    HIPCHK(hipMemcpyAsync(&a, dA, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&b, dB, 8, hipMemcpyDeviceToHost, s));
    if (dK) HIPCHK(hipMemcpyAsync(&k, dK, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (!(std::isfinite(a) && std::isfinite(b) && std::isfinite(k) && a >= 0 && b >= 0))
      return FRAM_EINVAL;
    perm_out[0] = 0;
    *objective_out = a * b + 2.0 * w * k;
  } else {
    NodeTerm nt;
    nt.K = dK;
    nt.w = dK ? w : 0.0;
    r = run_solve(c, L, dA, dB, nt, n, lambda, iters, tol, o, true, s, perm_out, objective_out,
                  &st);
  }
  st.ms_total = now_ms() - t0;
  c->last = st;
  if (stats) *stats = st;
  return r;
}

// ---------------------------------------------------------------------------
// Lockstep group of small pairs (fram_solve_many).  Every pair whose matrix
// is a single tile (n <= 256, edge 64, 128 or 256) runs Algorithm 1 in step
// with the others: each outer iteration is one launch per kernel for all
// active pairs (the two GEMMs, the whole SDSN projection -- statistics and
// every pass in one workgroup per pair --, the N update and delta), and one
// copy of all pairs' states back to the host, where each pair's stop rules
// are applied exactly as in run_solve; finished pairs leave the group.  Each
// job computes what the single-pair launch computes, so a pair's result
// equals, bit for bit, solving it alone with fram_options.tile set to its
// edge.  Small pairs on the single-pair path are bound by launch and
// host-synchronisation latency (two state reads per outer iteration); here
// the latency is shared by the whole group.

int group_edge(int n) { return n <= 64 ? 64 : (n <= 128 ? 128 : 256); }

bool group_eligible(int n, const fram_options& o) {
  return n >= 2 && n <= 256 && o.variant == 0 && o.stable_iters == 0 && o.profile == 0 &&
         o.sdsn_mode != 2 && (o.tile == 0 || o.tile == group_edge(n));
}

void shift_layout(Layout& L, size_t b) {
  for (size_t* f : {&L.A64, &L.B64, &L.K64, &L.Kp, &L.Alp, &L.Blp, &L.W, &L.N, &L.Nlp, &L.X,
                    &L.Nprev, &L.rowp[0], &L.rowp[1], &L.colp[0], &L.colp[1], &L.tot[0],
                    &L.tot[1], &L.tmax[0], &L.tmax[1], &L.upd, &L.mx, &L.obj, &L.sigma, &L.lap,
                    &L.state})
    *f += b;
}

fram_status solve_group(fram_ctx* c, const std::vector<int>& pairs, const double* const* A,
                        const double* const* B, const int* n, double theta, int iters,
                        double tol, const fram_options& o, int32_t* const* perm_out,
                        double* objective_out, fram_stats* stats) {
  const int G = (int)pairs.size();
  if (G == 0) return FRAM_OK;
  const Elem e = (Elem)o.prec;
  std::vector<Layout> Ls(G);
  size_t off = 0;
  for (int g = 0; g < G; ++g) {
    const int m = n[pairs[g]];
    Ls[g] = plan(m, e, group_edge(m), Use::Solve);
    shift_layout(Ls[g], off);
    off += align_up(Ls[g].total);
  }
  const size_t states_off = off;
  off += align_up((size_t)G * sizeof(DevState));
  const size_t jobs_off = off;
  const size_t jobs_bytes =
      (size_t)G * (2 * sizeof(fram::GemmJob) + sizeof(fram::SdsnJob) + sizeof(fram::UpdateJob));
  off += align_up(jobs_bytes);
  if (c->budget != 0 && off > c->budget) {
    c->err = "the group's workspace exceeds the HBM budget";
    return FRAM_ENOMEM;
  }
  fram_status r = ensure_device(c);
  if (r != FRAM_OK) return r;
  r = ensure_ws(c, off);
  if (r != FRAM_OK) return r;
  hipStream_t s = c->stream;
  DevState* states = at<DevState>(c, states_off);
  HIPCHK(fram::launch_zero(states, (size_t)G * sizeof(DevState), s));

  // Algorithm 1, steps 1-3 for every pair, as in run_solve.
  for (int g = 0; g < G; ++g) {
    const Layout& L = Ls[g];
    const int p = pairs[g], m = n[p];
    const size_t np2 = (size_t)L.np * L.np;
    double* dA = at<double>(c, L.A64);
    double* dB = at<double>(c, L.B64);
    HIPCHK(hipMemcpyAsync(dA, A[p], (size_t)m * m * 8, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dB, B[p], (size_t)m * m * 8, hipMemcpyHostToDevice, s));
    HIPCHK(fram::launch_maxes(dA, dB, m, at<double>(c, L.mx), L.nmax, &states[g], s));
    HIPCHK(fram::launch_cast_scaled(e, dA, m, at<void>(c, L.Alp), L.np, &states[g], 0, s));
    HIPCHK(fram::launch_cast_scaled(e, dB, m, at<void>(c, L.Blp), L.np, &states[g], 1, s));
    HIPCHK(fram::launch_zero(at<float>(c, L.N), np2 * 4, s));
    if (e != Elem::F32) HIPCHK(fram::launch_zero(at<void>(c, L.Nlp), np2 * fram::elem_size(e), s));
  }

  struct PairRun {
    int it = 0, total_passes = 0, last_passes = 0, max_passes = 0, stall = 0;
    bool capped = false, converged = false, stalled = false;
    double gamma = 0.0, delta = 0.0, dmin = 0.0;
  };
  std::vector<PairRun> run(G);
  std::vector<int> active(G);
  for (int g = 0; g < G; ++g) active[g] = g;
  std::vector<DevState> hs(G);
  std::vector<char> stage(jobs_bytes);
  char* djobs = at<char>(c, jobs_off);
  const bool watch_stall = o.stall_iters > 0;
  for (int it = 1; it <= iters && !active.empty(); ++it) {
    // Job tables of the active pairs: GEMM and SDSN jobs grouped by edge,
    // update jobs for all.
    const int A_ = (int)active.size();
    fram::GemmJob* g1 = reinterpret_cast<fram::GemmJob*>(stage.data());
    fram::GemmJob* g2 = g1 + A_;
    fram::SdsnJob* sj = reinterpret_cast<fram::SdsnJob*>(g2 + A_);
    fram::UpdateJob* uj = reinterpret_cast<fram::UpdateJob*>(sj + A_);
    int cnt[3] = {0, 0, 0}, first[3] = {0, 0, 0};
    std::vector<int> order;
    order.reserve(A_);
    for (int k = 0; k < 3; ++k) {
      first[k] = (int)order.size();
      for (int g : active)
        if (group_edge(n[pairs[g]]) == (64 << k)) order.push_back(g);
      cnt[k] = (int)order.size() - first[k];
    }
    int max_blocks = 1;
    for (int q = 0; q < A_; ++q) {
      const int g = order[q];
      const Layout& L = Ls[g];
      const int m = n[pairs[g]];
      void* Nlp = (e == Elem::F32) ? at<void>(c, L.N) : at<void>(c, L.Nlp);
      g1[q] = {at<void>(c, L.Blp), Nlp, at<void>(c, L.W), L.np, fram::gemm_ktiles(e, m)};
      g2[q] = {at<void>(c, L.Alp), at<void>(c, L.W), at<void>(c, L.X), L.np,
               fram::gemm_ktiles(e, m)};
      sj[q] = {at<float>(c, L.X), m, L.np, partials(c, L, 0), partials(c, L, 1), &states[g]};
      uj[q] = {at<float>(c, L.X), at<float>(c, L.N), Nlp, m, L.np, L.nupd, at<double>(c, L.upd),
               &states[g]};
      max_blocks = std::max(max_blocks, L.nupd);
    }
    const size_t used = (size_t)A_ * (2 * sizeof(fram::GemmJob) + sizeof(fram::SdsnJob) +
                                      sizeof(fram::UpdateJob));
    // The tables are rewritten each iteration after the previous iteration's
    // launches have finished (the state copy below synchronises).
    HIPCHK(hipMemcpyAsync(djobs, stage.data(), used, hipMemcpyHostToDevice, s));
    const fram::GemmJob* d1 = reinterpret_cast<const fram::GemmJob*>(djobs);
    const fram::GemmJob* d2 = d1 + A_;
    const fram::SdsnJob* ds = reinterpret_cast<const fram::SdsnJob*>(d2 + A_);
    const fram::UpdateJob* du = reinterpret_cast<const fram::UpdateJob*>(ds + A_);
    for (int k = 0; k < 3; ++k)  // Step 5: W = B N^T, X = A W^T
      HIPCHK(fram::launch_gemm_group(e, 64 << k, false, d1 + first[k], cnt[k], s));
    for (int k = 0; k < 3; ++k)
      HIPCHK(fram::launch_gemm_group(e, 64 << k, true, d2 + first[k], cnt[k], s));
    for (int k = 0; k < 3; ++k)  // Step 6: D = SDSN(X, theta)
      HIPCHK(fram::launch_sdsn_group(64 << k, ds + first[k], cnt[k], o.sdsn_max, theta,
                                     o.gamma_tol, s));
    // Steps 7-8: N update and delta.
    HIPCHK(fram::launch_update_group(e, du, A_, max_blocks, o.alpha, s));
    HIPCHK(hipMemcpyAsync(hs.data(), states, (size_t)G * sizeof(DevState),
                          hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int> still;
    still.reserve(A_);
    for (int g : active) {
      PairRun& pr = run[g];
      const DevState& h = hs[g];
      const int p = pairs[g];
      pr.it = it;
      if (!h.done) {
        c->err = "pair " + std::to_string(p) + ": SDSN loop ended without completion flag";
        return FRAM_EDEVICE;
      }
      pr.gamma = h.gamma;
      pr.total_passes += h.passes;
      pr.last_passes = h.passes;
      pr.max_passes = std::max(pr.max_passes, h.passes);
      pr.capped = pr.capped || ((h.passes >= o.sdsn_max) && !(h.gamma <= o.gamma_tol));
      if (!std::isfinite(h.gamma)) {
        c->err = "pair " + std::to_string(p) + ": non-finite gamma in SDSN";
        return FRAM_ENUMERIC;
      }
      bool finished = it == iters;
      if (tol > 0.0 || watch_stall || it == iters) {
        pr.delta = h.delta;
        if (!std::isfinite(pr.delta)) {
          c->err = "pair " + std::to_string(p) + ": non-finite delta";
          return FRAM_ENUMERIC;
        }
        if (pr.delta <= tol) {
          pr.converged = true;
          finished = true;
        } else if (watch_stall && pr.delta <= o.stall_delta) {
          pr.stall = (pr.dmin > 0.0 && pr.delta >= pr.dmin) ? pr.stall + 1 : 0;
          pr.dmin = (pr.dmin > 0.0) ? std::min(pr.dmin, pr.delta) : pr.delta;
          if (pr.stall >= o.stall_iters) {
            pr.converged = true;
            pr.stalled = true;
            finished = true;
          }
        }
      }
      if (!finished) still.push_back(g);
    }
    active.swap(still);
  }

  // Step 10 and the objective, pair by pair (as run_solve does).
  Prof prof{0, c, s, 0.0f};
  for (int g = 0; g < G; ++g) {
    const Layout& L = Ls[g];
    const int p = pairs[g], m = n[p];
    fram_stats st{};
    int lap_paths = 0;
    r = finish_discretise(c, L, m, at<double>(c, L.A64), at<double>(c, L.B64), NodeTerm{},
                          at<float>(c, L.N), at<int32_t>(c, L.sigma), &states[g], s, perm_out[p],
                          &objective_out[p], &lap_paths, prof, &st);
    if (r != FRAM_OK) {
      c->err = "pair " + std::to_string(p) + ": " + c->err;
      return r;
    }
    const PairRun& pr = run[g];
    st.outer_iters = pr.it;
    st.sdsn_passes = pr.total_passes;
    st.sdsn_passes_last = pr.last_passes;
    st.sdsn_passes_max = pr.max_passes;
    st.converged = pr.converged ? 1 : 0;
    st.sdsn_capped = pr.capped ? 1 : 0;
    st.lap_paths = lap_paths;
    st.stalled = pr.stalled ? 1 : 0;
    st.gemm_tile = L.bm;
    st.delta = pr.delta;
    st.gamma = pr.gamma;
    if (stats) stats[p] = st;
  }
  return FRAM_OK;
}

}  // namespace

// ============================================================================ C ABI
extern "C" {

void fram_struct_sizes(size_t* options_bytes, size_t* stats_bytes) {
  if (options_bytes) *options_bytes = sizeof(fram_options);
  if (stats_bytes) *stats_bytes = sizeof(fram_stats);
}

void fram_default_options(fram_options* opt) {
  if (!opt) return;
  opt->prec = FRAM_FP32;
  opt->alpha = 0.95;
  opt->gamma_tol = 1e-6;
  opt->sdsn_max = 1000;
  opt->tile = 0;
  opt->profile = 0;
  opt->sdsn_mode = 0;
  opt->stable_iters = 0;
  opt->stall_iters = 0;
  opt->stall_delta = 1e-3;
  opt->variant = 0;
  opt->dsn_iters = 30;
  opt->many_workers = 16;
  opt->N0 = nullptr;
  opt->N_out = nullptr;
  opt->onchip_roll_us = 0;
  opt->onchip_barrier_us = 0;
}

fram_status fram_create(fram_ctx** out, int device, size_t hbm_budget_bytes) {
  if (!out || device < 0) return FRAM_EINVAL;
  fram_ctx* c = new (std::nothrow) fram_ctx();
  if (!c) return FRAM_ENOMEM;
  c->device = device;
  c->budget = hbm_budget_bytes;
  *out = c;
  return FRAM_OK;
}

void fram_destroy(fram_ctx* c) {
  if (!c) return;
  for (fram_ctx* w : c->workers) fram_destroy(w);
  if (c->group) fram_destroy(c->group);
  if (c->inited) {
    for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->ws) (void)hipFree(c->ws);
    if (c->hst) (void)hipHostFree(c->hst);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->sync) (void)hipFree(c->sync);
    if (c->stream) (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

size_t fram_resident_bytes(const fram_ctx* c) {
  if (!c) return 0;
  size_t b = c->ws_bytes + (c->sync ? fram::kOnchipSyncBytes : 0);
  for (const fram_ctx* w : c->workers) b += fram_resident_bytes(w);
  if (c->group) b += fram_resident_bytes(c->group);
  return b;
}

fram_status fram_trim(fram_ctx* c) {
  if (!c) return FRAM_OK;
  for (fram_ctx* w : c->workers) {
    const fram_status r = fram_trim(w);
    if (r != FRAM_OK) return r;
  }
  if (c->group) {
    const fram_status r = fram_trim(c->group);
    if (r != FRAM_OK) return r;
  }
  if (c->ws) {
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  return FRAM_OK;
}

fram_status fram_set_tile_table(const int* n_max, const int* tile, int count) {
  if (count < 0 || count > kMaxTileBuckets) return FRAM_EINVAL;
  if (count > 0 && (!n_max || !tile)) return FRAM_EINVAL;
  for (int k = 0; k < count; ++k) {
    if (n_max[k] < 1 || (k > 0 && n_max[k] <= n_max[k - 1])) return FRAM_EINVAL;
    if (tile[k] != 64 && tile[k] != 128 && tile[k] != 256) return FRAM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_tile_mu);
  for (int k = 0; k < count; ++k) {
    g_tile_nmax[k] = n_max[k];
    g_tile_edge[k] = tile[k];
  }
  g_tile_count = count;
  return FRAM_OK;
}

int fram_auto_tile(int n) {
  if (n < 1 || n > FRAM_MAX_N) return 0;
  return choose_tile(n, 0);
}

size_t fram_workspace_bytes(int n, fram_precision prec, int tile) {
  if (n < 1 || n > FRAM_MAX_N || !valid_prec((int)prec)) return 0;
  return plan(n, (Elem)prec, tile, Use::Solve).total;
}

fram_status fram_solve_ex(fram_ctx* c, const double* A, const double* B, int n, double lambda,
                          int iters, double tol, const fram_options* opt, int32_t* perm_out,
                          double* objective_out, fram_stats* stats) {
  if (!c || !A || !B || !perm_out || !objective_out) return FRAM_EINVAL;
  fram_options o = opt ? *opt : defaults();
  fram_status r = check_options(o);
  if (r == FRAM_OK) r = check_scalars(n, lambda, iters, tol);
  if (r == FRAM_OK) r = check_graph(A, n);
  if (r == FRAM_OK) r = check_graph(B, n);
  if (r == FRAM_OK) r = check_warm(o, n);
  if (r != FRAM_OK) {
    c->err = "invalid argument";
    return r;
  }
  fram_stats st{};
  r = solve_host_impl(c, A, B, nullptr, 0.0, n, lambda, iters, tol, o, perm_out, objective_out,
                      &st);
  c->last = st;
  if (stats) *stats = st;
  return r;
}

fram_status fram_solve(fram_ctx* c, const double* A, const double* B, int n, double lambda,
                       int iters, double tol, int32_t* perm_out, double* objective_out) {
  return fram_solve_ex(c, A, B, n, lambda, iters, tol, nullptr, perm_out, objective_out,
                       nullptr);
}

fram_status fram_solve_dev(fram_ctx* c, const double* dA, const double* dB, int n,
                           double lambda, int iters, double tol, const fram_options* opt,
                           int32_t* perm_out, double* objective_out, fram_stats* stats,
                           void* stream) {
  if (!c || !dA || !dB || !perm_out || !objective_out) return FRAM_EINVAL;
  fram_options o = opt ? *opt : defaults();
  fram_status r = check_options(o);
  if (r == FRAM_OK) r = check_scalars(n, lambda, iters, tol);
  if (r != FRAM_OK) {
    c->err = "invalid argument";
    return r;
  }
  return solve_dev_impl(c, dA, dB, nullptr, 0.0, n, lambda, iters, tol, o, perm_out,
                        objective_out, stats, stream);
}

fram_status fram_solve_attr_ex(fram_ctx* c, const double* A, const double* B, const double* K,
                               int n, double node_weight, double lambda, int iters, double tol,
                               const fram_options* opt, int32_t* perm_out, double* objective_out,
                               fram_stats* stats) {
  if (!c || !A || !B || !K || !perm_out || !objective_out) return FRAM_EINVAL;
  fram_options o = opt ? *opt : defaults();
  fram_status r = check_options(o);
  if (r == FRAM_OK && o.variant != 0) r = FRAM_EINVAL;  // DSPFP has no node term here
  if (r == FRAM_OK) r = check_scalars(n, lambda, iters, tol);
  if (r == FRAM_OK) r = check_graph(A, n);
  if (r == FRAM_OK) r = check_graph(B, n);
  if (r == FRAM_OK && !std::isfinite(node_weight)) r = FRAM_EINVAL;
  for (size_t t = 0; r == FRAM_OK && t < (size_t)n * n; ++t)
    if (!std::isfinite(K[t])) r = FRAM_EINVAL;
  if (r == FRAM_OK) r = check_warm(o, n);
  if (r != FRAM_OK) {
    c->err = "invalid argument";
    return r;
  }
  fram_stats st{};
  r = solve_host_impl(c, A, B, K, node_weight, n, lambda, iters, tol, o, perm_out, objective_out,
                      &st);
  c->last = st;
  if (stats) *stats = st;
  return r;
}

fram_status fram_solve_attr_dev(fram_ctx* c, const double* dA, const double* dB,
                                const double* dK, int n, double node_weight, double lambda,
                                int iters, double tol, const fram_options* opt, int32_t* perm_out,
                                double* objective_out, fram_stats* stats, void* stream) {
  if (!c || !dA || !dB || !dK || !perm_out || !objective_out) return FRAM_EINVAL;
  fram_options o = opt ? *opt : defaults();
  fram_status r = check_options(o);
  if (r == FRAM_OK && o.variant != 0) r = FRAM_EINVAL;  // DSPFP has no node term here
  if (r == FRAM_OK) r = check_scalars(n, lambda, iters, tol);
  if (r == FRAM_OK && !std::isfinite(node_weight)) r = FRAM_EINVAL;
  if (r != FRAM_OK) {
    c->err = "invalid argument";
    return r;
  }
  return solve_dev_impl(c, dA, dB, dK, node_weight, n, lambda, iters, tol, o, perm_out,
                        objective_out, stats, stream);
}

fram_status fram_sdsn_project_dev(fram_ctx* c, const float* dK, int ldk, int n, double lambda,
                                  const fram_options* opt, float* dX, int ldx,
                                  fram_stats* stats, void* stream) {
  if (!c || !dK || !dX) return FRAM_EINVAL;
  fram_options o = opt ? *opt : defaults();
  fram_status r = check_options(o);
  if (r != FRAM_OK || n < 1 || n > FRAM_MAX_N || ldk < n || ldx < n || ldk > FRAM_MAX_N ||
      ldx > FRAM_MAX_N || !(lambda > 0.0) || !std::isfinite(lambda)) {
    c->err = "invalid argument";
    return FRAM_EINVAL;
  }
  const double t0 = now_ms();
  const Layout L = plan(n, Elem::F32, o.tile, Use::Sdsn);
  if (c->budget != 0 && L.total > c->budget) {
    c->err = "workspace exceeds the HBM budget";
    return FRAM_ENOMEM;
  }
  r = ensure_device(c);
  if (r != FRAM_OK) return r;
  r = ensure_ws(c, L.total);
  if (r != FRAM_OK) return r;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  DevState* st = at<DevState>(c, L.state);
  float* X = at<float>(c, L.X);
  c->pending.clear();
  c->evused = 0;
  HIPCHK(fram::launch_zero(st, sizeof(DevState), s));
  int passes = 0;
  double gamma = 0.0;
  bool capped = false;
  fram_stats stt{};
  bool onchip = false;
  r = use_onchip(c, L, o, &onchip);
  if (r != FRAM_OK) return r;
  bool streamed = !onchip;
  if (onchip) {
    Prof prof{o.profile, c, s, 0.0f};
    r = timed(prof, &stt.ms_sdsn, nullptr, [&] {
      fram_status q = run_sdsn_onchip(c, L, n, dK, ldk, X, nullptr, nullptr, Elem::F32, 0.95, st,
                                      lambda, o, s);
      return q == FRAM_OK ? hipSuccess : hipErrorUnknown;
    });
    if (r != FRAM_OK) return r;
    r = read_state(c, st, s);
    if (r != FRAM_OK) return r;
    if (c->hst->invalid & (fram::kInvalidRollCall | fram::kInvalidBarrier)) {
      // Nothing was written (the input is untouched): stream instead.
      HIPCHK(fram::launch_zero(&st->invalid, sizeof(int), s));
      stt.sdsn_fallbacks = 1;
      streamed = true;
    } else {
      passes = c->hst->passes;
      gamma = c->hst->gamma;
      capped = passes >= o.sdsn_max && !(gamma <= o.gamma_tol);
      stt.sdsn_launches = 1;
      stt.sdsn_onchip = 1;
      if (!std::isfinite(gamma)) {
        c->err = "non-finite gamma in SDSN";
        return FRAM_ENUMERIC;
      }
    }
  }
  if (streamed) {
    HIPCHK(fram::launch_tile_stats(L.bm, dK, ldk, X, n, L.np, partials(c, L, 0), st, s));
    r = run_sdsn_passes(c, L, n, X, st, lambda, o, 8, s, &passes, &gamma, &capped, &stt);
    if (r != FRAM_OK) return r;
  }
  HIPCHK(fram::launch_copy_f32(X, L.np, dX, ldx, n, s));
  HIPCHK(hipStreamSynchronize(s));
  r = flush_timings(c);
  if (r != FRAM_OK) return r;
  if (o.profile == 2) stt.sdsn_launches = streamed ? passes : 1;
  stt.sdsn_passes = passes;
  stt.sdsn_passes_last = passes;
  stt.sdsn_passes_max = passes;
  stt.sdsn_capped = capped ? 1 : 0;
  stt.gamma = gamma;
  stt.gemm_tile = L.bm;
  stt.ms_total = now_ms() - t0;
  c->last = stt;
  if (stats) *stats = stt;
  return FRAM_OK;
}

fram_status fram_sdsn_project_ex(fram_ctx* c, const float* K, int n, double lambda,
                                 const fram_options* opt, float* X_out, fram_stats* stats) {
  if (!c || !K || !X_out || n < 1 || n > FRAM_MAX_N) return FRAM_EINVAL;
  fram_options o = opt ? *opt : defaults();
  if (check_options(o) != FRAM_OK || !(lambda > 0.0) || !std::isfinite(lambda)) return FRAM_EINVAL;
  for (size_t t = 0; t < (size_t)n * n; ++t)
    if (!std::isfinite(K[t])) return FRAM_EINVAL;
  const Layout L = plan(n, Elem::F32, o.tile, Use::Sdsn);
  const size_t extra = align_up((size_t)n * n * 4);
  if (c->budget != 0 && L.total + extra > c->budget) {
    c->err = "workspace exceeds the HBM budget";
    return FRAM_ENOMEM;
  }
  fram_status r = ensure_device(c);
  if (r != FRAM_OK) return r;
  r = ensure_ws(c, L.total + extra);
  if (r != FRAM_OK) return r;
  // The staging copy of K sits after the SDSN layout in the same workspace.
  float* dK = at<float>(c, L.total);
  HIPCHK(hipMemcpyAsync(dK, K, (size_t)n * n * 4, hipMemcpyHostToDevice, c->stream));
  r = fram_sdsn_project_dev(c, dK, n, n, lambda, &o, dK, n, stats, c->stream);
  if (r != FRAM_OK) return r;
  HIPCHK(hipMemcpyAsync(X_out, dK, (size_t)n * n * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return FRAM_OK;
}

fram_status fram_sdsn_project(fram_ctx* c, const float* K, int n, double lambda, float* X_out) {
  return fram_sdsn_project_ex(c, K, n, lambda, nullptr, X_out, nullptr);
}

fram_status fram_gradient(fram_ctx* c, const float* A, const float* N, const float* B, int n,
                          fram_precision prec, float* X_out) {
  if (!c || !A || !N || !B || !X_out || n < 1 || n > FRAM_MAX_N || !valid_prec((int)prec))
    return FRAM_EINVAL;
  const Elem e = (Elem)prec;
  const Layout L = plan(n, e, 0, Use::Gradient);
  if (c->budget != 0 && L.total > c->budget) {
    c->err = "workspace exceeds the HBM budget";
    return FRAM_ENOMEM;
  }
  fram_status r = ensure_device(c);
  if (r != FRAM_OK) return r;
  r = ensure_ws(c, L.total);
  if (r != FRAM_OK) return r;
  hipStream_t s = c->stream;
  float* X = at<float>(c, L.X);
  float* N32 = at<float>(c, L.N);
  void* Alp = at<void>(c, L.Alp);
  void* Blp = at<void>(c, L.Blp);
  void* W = at<void>(c, L.W);
  void* Nlp = (e == Elem::F32) ? (void*)N32 : at<void>(c, L.Nlp);
  const size_t bytes = (size_t)n * n * 4;
  // Stage each host operand through X (n*n floats fit in np*np), then cast.
  HIPCHK(hipMemcpyAsync(X, A, bytes, hipMemcpyHostToDevice, s));
  HIPCHK(fram::launch_cast_f32(e, X, n, Alp, L.np, s));
  HIPCHK(hipMemcpyAsync(X, B, bytes, hipMemcpyHostToDevice, s));
  HIPCHK(fram::launch_cast_f32(e, X, n, Blp, L.np, s));
  HIPCHK(hipMemcpyAsync(X, N, bytes, hipMemcpyHostToDevice, s));
  HIPCHK(fram::launch_cast_f32(e, X, n, Nlp, L.np, s));
  HIPCHK(fram::launch_gemm_nt(e, L.bm, Blp, Nlp, W, false, n, L.np, L.np, s));
  HIPCHK(fram::launch_gemm_nt(e, L.bm, Alp, W, X, true, n, L.np, L.np, s));
  HIPCHK(hipMemcpy2DAsync(X_out, (size_t)n * 4, X, (size_t)L.np * 4, (size_t)n * 4, n,
                          hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return FRAM_OK;
}

}  // extern "C"

extern "C" {

fram_status fram_solve_many_ex(fram_ctx* c, int count, const double* const* A,
                               const double* const* B, const int* n, double lambda, int iters,
                               double tol, const fram_options* opt, int32_t* const* perm_out,
                               double* objective_out, fram_stats* stats) {
  if (!c || count < 1 || !A || !B || !n || !perm_out || !objective_out) return FRAM_EINVAL;
  fram_options o = opt ? *opt : defaults();
  if (!opt) o.prec = FRAM_BF16;
  fram_status r = check_options(o);
  if (r != FRAM_OK) return r;
  if (o.N0 != nullptr || o.N_out != nullptr) {
    c->err = "fram_solve_many takes no warm start or final iterate";
    return FRAM_EINVAL;
  }
  for (int p = 0; p < count; ++p) {
    if (!A[p] || !B[p] || !perm_out[p]) return FRAM_EINVAL;
    r = check_scalars(n[p], lambda, iters, tol);
    if (r == FRAM_OK) r = check_graph(A[p], n[p]);
    if (r == FRAM_OK) r = check_graph(B[p], n[p]);
    if (r != FRAM_OK) {
      c->err = "invalid argument in pair " + std::to_string(p);
      return r;
    }
  }
  const double t0 = now_ms();
  std::vector<int> single;
  for (int p = 0; p < count; ++p) {
    if (n[p] == 1) {
      perm_out[p][0] = 0;
      objective_out[p] = A[p][0] * B[p][0];
      if (stats) stats[p] = fram_stats{};
    } else {
      single.push_back(p);
    }
  }
  // Pairs whose matrix is a single tile run in the lockstep group (its own
  // context and host thread); the others run the single-pair path, up to
  // o.many_workers pairs at a time, each on a worker context with its own
  // stream and workspace (one host thread per worker), largest pairs first.
  // Nothing is shared between the group and the workers but the device.
  std::vector<int> grouped, rest;
  for (int p : single) (group_eligible(n[p], o) ? grouped : rest).push_back(p);
  single.swap(rest);
  std::thread group_thread;
  fram_status group_status = FRAM_OK;
  if (!grouped.empty()) {
    if (c->group == nullptr) {
      r = fram_create(&c->group, c->device, c->budget == 0 ? 0 : c->budget / 2);
      if (r != FRAM_OK) return r;
    }
    group_thread = std::thread([&] {
      group_status = solve_group(c->group, grouped, A, B, n, lambda, iters, tol, o, perm_out,
                                 objective_out, stats);
    });
  }
  if (!single.empty()) {
    std::stable_sort(single.begin(), single.end(), [&](int x, int y) { return n[x] > n[y]; });
    const int nw = (int)std::min<size_t>((size_t)o.many_workers, single.size());
    while ((int)c->workers.size() < nw) {
      fram_ctx* w = nullptr;
      // The context's HBM budget is shared out evenly between its workers.
      r = fram_create(&w, c->device, c->budget == 0 ? 0 : c->budget / kMaxManyWorkers);
      if (r != FRAM_OK) return r;
      c->workers.push_back(w);
    }
    std::atomic<int> next{0};
    std::atomic<int> failed{0};
    std::mutex mu;
    fram_status first = FRAM_OK;
    auto work = [&](fram_ctx* w) {
      while (!failed.load()) {
        const int q = next.fetch_add(1);
        if (q >= (int)single.size()) return;
        const int p = single[q];
        fram_stats st{};
        const fram_status rr = solve_host_impl(w, A[p], B[p], nullptr, 0.0, n[p], lambda, iters,
                                               tol, o, perm_out[p], &objective_out[p], &st);
        if (stats) stats[p] = st;
        if (rr != FRAM_OK) {
          std::lock_guard<std::mutex> lk(mu);
          if (first == FRAM_OK) {
            first = rr;
            c->err = "pair " + std::to_string(p) + ": " + w->err;
          }
          failed.store(1);
          return;
        }
      }
    };
    if (nw == 1) {
      work(c->workers[0]);
    } else {
      std::vector<std::thread> th;
      for (int t = 0; t < nw; ++t) th.emplace_back(work, c->workers[t]);
      for (auto& t : th) t.join();
    }
    if (first != FRAM_OK) {
      if (group_thread.joinable()) group_thread.join();
      return first;
    }
  }
  if (group_thread.joinable()) group_thread.join();
  if (group_status != FRAM_OK) {
    c->err = "lockstep group: " + c->group->err;
    return group_status;
  }
  const double ms = now_ms() - t0;
  if (stats)
    for (int p = 0; p < count; ++p) stats[p].ms_total = ms;
  c->last = stats ? stats[count - 1] : fram_stats{};
  c->last.ms_total = ms;
  return FRAM_OK;
}

fram_status fram_solve_many(fram_ctx* c, int count, const double* const* A,
                            const double* const* B, const int* n, double lambda, int iters,
                            double tol, int32_t* const* perm_out, double* objective_out) {
  return fram_solve_many_ex(c, count, A, B, n, lambda, iters, tol, nullptr, perm_out,
                            objective_out, nullptr);
}

namespace {

// Workspace of the assignment entry points: the assignment's arrays, then
// the device state.
size_t assign_ws_bytes(int n) {
  return align_up(fram::lap_workspace_bytes(n)) + align_up(sizeof(DevState));
}

// Device assignment of an n x n FP32 matrix at dW (leading dimension ldw)
// into dperm on stream s, then a check that the result is a permutation.
fram_status assign_on_device(fram_ctx* c, const float* dW, int ldw, int n, int32_t* dperm,
                             hipStream_t s, int32_t* host_perm) {
  const size_t st_off = align_up(fram::lap_workspace_bytes(n));
  fram_status r = ensure_ws(c, assign_ws_bytes(n));
  if (r != FRAM_OK) return r;
  char* lws = at<char>(c, 0);
  DevState* st = at<DevState>(c, st_off);
  double* u = reinterpret_cast<double*>(lws);
  HIPCHK(fram::launch_zero(st, sizeof(DevState), s));
  HIPCHK(fram::launch_row_argmax(dW, n, ldw, dperm, s, u));
  fram::LapProblem lp{dW, n, ldw, dperm, lws, u, 1, &st->lap_paths};
  HIPCHK(fram::launch_lap(&lp, nullptr, 1, n, s));
  HIPCHK(hipMemcpyAsync(host_perm, dperm, (size_t)n * 4, hipMemcpyDeviceToHost, s));
  r = read_state(c, st, s);
  if (r != FRAM_OK) return r;
  c->last = fram_stats{};
  c->last.lap_paths = c->hst->lap_paths;
  if (!is_permutation(host_perm, n)) {
    c->err = "no finite assignment (non-finite entries)";
    return FRAM_ENUMERIC;
  }
  return FRAM_OK;
}

}  // namespace

fram_status fram_assign(fram_ctx* c, const float* W, int n, int32_t* perm_out) {
  if (!c || !W || !perm_out || n < 1 || n > FRAM_MAX_N) return FRAM_EINVAL;
  for (size_t t = 0; t < (size_t)n * n; ++t)
    if (!std::isfinite(W[t])) return FRAM_EINVAL;
  const size_t wbytes = align_up((size_t)n * n * 4);
  const size_t base = assign_ws_bytes(n);
  if (c->budget != 0 && base + wbytes + align_up((size_t)n * 4) > c->budget) {
    c->err = "workspace exceeds the HBM budget";
    return FRAM_ENOMEM;
  }
  fram_status r = ensure_device(c);
  if (r != FRAM_OK) return r;
  r = ensure_ws(c, base + wbytes + align_up((size_t)n * 4));
  if (r != FRAM_OK) return r;
  hipStream_t s = c->stream;
  float* dW = at<float>(c, base);
  int32_t* dp = at<int32_t>(c, base + wbytes);
  HIPCHK(hipMemcpyAsync(dW, W, (size_t)n * n * 4, hipMemcpyHostToDevice, s));
  return assign_on_device(c, dW, n, n, dp, s, perm_out);
}

fram_status fram_assign_dev(fram_ctx* c, const float* dW, int ldw, int n, int32_t* dperm,
                            void* stream) {
  if (!c || !dW || !dperm || n < 1 || n > FRAM_MAX_N || ldw < n || ldw > FRAM_MAX_N)
    return FRAM_EINVAL;
  fram_status r = ensure_device(c);
  if (r != FRAM_OK) return r;
  hipStream_t s = stream ? static_cast<hipStream_t>(stream) : c->stream;
  std::vector<int32_t> host(n);
  return assign_on_device(c, dW, ldw, n, dperm, s, host.data());
}

fram_status fram_last_stats(const fram_ctx* c, fram_stats* out) {
  if (!c || !out) return FRAM_EINVAL;
  *out = c->last;
  return FRAM_OK;
}

const char* fram_status_str(fram_status s) {
  switch (s) {
    case FRAM_OK:
      return "ok";
    case FRAM_EINVAL:
      return "invalid argument";
    case FRAM_ENOMEM:
      return "out of HBM budget";
    case FRAM_EDEVICE:
      return "device error";
    case FRAM_ENUMERIC:
      return "non-finite value";
    case FRAM_EBUSY:
      return "busy";
  }
  return "unknown status";
}

const char* fram_last_error(const fram_ctx* c) { return c ? c->err.c_str() : ""; }

}  // extern "C"
