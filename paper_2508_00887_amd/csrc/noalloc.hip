// fram_sdsn_project_noalloc: the SDSN projection (Algorithm 2) for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// It runs the streaming passes of fram_sdsn_project_dev (the same kernels, so
// the same iterates bit for bit) with their working memory -- the padded
// iterate, two sets of tile partials and the device state -- in a file-scope
// device array instead of a context workspace.  No context is involved, so
// nothing else is allocated either: no stream, event or pinned host buffer.
// The array is resolved to a device address once per device, on the first
// call made with that device current, and that address (never the array's
// name, which in host code only stands in for the symbol) is what the kernels
// receive.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/fram.h"
#include "fram_internal.h"

namespace fram {
namespace {

// Working memory of one projection of size n <= FRAM_NOALLOC_MAX_N:
// n <= 64 is one 64-tile, n <= 128 one 128-tile, larger sizes use 64-tiles
// (np <= 1024): the padded iterate (np^2 floats) and two partial sets.
constexpr size_t kScratchBytes = 6u << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

struct NoallocLayout {
  int bm, np, nb;
  size_t X, rowp[2], colp[2], tot[2], tmax[2], state, total;
};

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

NoallocLayout plan_noalloc(int n, int tile) {
  NoallocLayout L{};
  L.bm = (tile == 64 || tile == 128) ? tile : (n > 64 && n <= 128 ? 128 : 64);
  L.np = (n + L.bm - 1) / L.bm * L.bm;
  L.nb = L.np / L.bm;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off += align256(bytes);
    return at;
  };
  L.X = take((size_t)L.np * L.np * 4);
  for (int k = 0; k < 2; ++k) {
    L.rowp[k] = take((size_t)L.nb * L.np * 8);
    L.colp[k] = take((size_t)L.nb * L.np * 8);
    L.tot[k] = take((size_t)L.nb * L.nb * 8);
    L.tmax[k] = take((size_t)L.nb * L.nb * 4);
  }
  L.state = take(sizeof(DevState));
  L.total = off;
  return L;
}

// Device address of `scratch` on the current device (looked up once).
hipError_t scratch_ptr(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

Partials partials_at(unsigned char* base, const NoallocLayout& L, int k) {
  Partials p;
  p.rowp = reinterpret_cast<double*>(base + L.rowp[k]);
  p.colp = reinterpret_cast<double*>(base + L.colp[k]);
  p.tot = reinterpret_cast<double*>(base + L.tot[k]);
  p.tmax = reinterpret_cast<float*>(base + L.tmax[k]);
  return p;
}

}  // namespace
}  // namespace fram

extern "C" fram_status fram_sdsn_project_noalloc(const float* dK, int ldk, int n, double lambda,
                                                 const fram_options* opt, float* dX, int ldx,
                                                 fram_stats* stats, void* stream) {
  using namespace fram;
  fram_options o;
  fram_default_options(&o);
  if (opt) o = *opt;
  if (!dK || !dX || n < 1 || n > FRAM_NOALLOC_MAX_N || ldk < n || ldx < n) return FRAM_EINVAL;
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return FRAM_EINVAL;
  if (!(o.gamma_tol >= 0.0) || !std::isfinite(o.gamma_tol) || o.sdsn_max < 1) return FRAM_EINVAL;
  if (o.sdsn_mode == 2 || o.sdsn_mode < 0 || o.sdsn_mode > 2) return FRAM_EINVAL;
  if (!(o.tile == 0 || o.tile == 64 || o.tile == 128)) return FRAM_EINVAL;
  const NoallocLayout L = plan_noalloc(n, o.tile);
  if (L.total > kScratchBytes) return FRAM_EINVAL;
  unsigned char* base = nullptr;
  if (scratch_ptr(&base) != hipSuccess) return FRAM_EDEVICE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float* X = reinterpret_cast<float*>(base + L.X);
  DevState* st = reinterpret_cast<DevState*>(base + L.state);
  DevState h{};
  auto read_state = [&]() {
    if (hipMemcpyAsync(&h, st, sizeof(DevState), hipMemcpyDeviceToHost, s) != hipSuccess)
      return false;
    return hipStreamSynchronize(s) == hipSuccess;
  };
  // The scratch array keeps the previous call's contents: the state starts
  // from zero, and the statistics pass rewrites the iterate (with its zero
  // padding) and the first partial set.
  if (launch_zero(st, sizeof(DevState), s) != hipSuccess) return FRAM_EDEVICE;
  if (launch_tile_stats(L.bm, dK, ldk, X, n, L.np, partials_at(base, L, 0), st, s) != hipSuccess)
    return FRAM_EDEVICE;
  const int last = o.sdsn_max + 1;  // the pass index that only evaluates gamma
  if (L.nb == 1) {
    if (launch_sdsn_chunk(L.bm, X, n, L.np, partials_at(base, L, 0), partials_at(base, L, 1), st,
                          1, last, o.sdsn_max, lambda, o.gamma_tol, s) != hipSuccess)
      return FRAM_EDEVICE;
    if (!read_state()) return FRAM_EDEVICE;
  } else {
    int k = 1, chunk = 8;
    while (true) {
      const int end = k + chunk - 1 < last ? k + chunk - 1 : last;
      for (int kk = k; kk <= end; ++kk)
        if (launch_sdsn_pass(L.bm, X, n, L.np, partials_at(base, L, (kk - 1) & 1),
                             partials_at(base, L, kk & 1), st, kk, o.sdsn_max, lambda,
                             o.gamma_tol, s) != hipSuccess)
          return FRAM_EDEVICE;
      k = end + 1;
      if (!read_state()) return FRAM_EDEVICE;
      if (h.done || k > last) break;
      chunk = 16;
    }
  }
  if (!h.done) return FRAM_EDEVICE;
  if (!std::isfinite(h.gamma)) return FRAM_ENUMERIC;
  if (launch_copy_f32(X, L.np, dX, ldx, n, s) != hipSuccess) return FRAM_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return FRAM_EDEVICE;
  if (stats) {
    fram_stats r{};
    r.outer_iters = 0;
    r.sdsn_passes = r.sdsn_passes_last = r.sdsn_passes_max = h.passes;
    r.sdsn_capped = (h.passes >= o.sdsn_max && !(h.gamma <= o.gamma_tol)) ? 1 : 0;
    r.gamma = h.gamma;
    r.gemm_tile = L.bm;
    *stats = r;
  }
  return FRAM_OK;
}
