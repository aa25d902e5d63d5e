// Launcher of the device linear assignment (lap_device.h): one workgroup per
// problem.  Its arrays live in LDS when they fit (n <= 4400), else in the
// problem's global workspace; the unmatched-row list is always in the
// workspace, after the arrays.
#include "lap_device.h"

namespace fram {
namespace {

constexpr size_t kLapLdsBytes = 160 * 1024 - 1024;  // minus the static LDS

template <int NT, bool IN_LDS>
__global__ __launch_bounds__(NT) void lap_kernel(LapProblem one,
                                                 const LapProblem* __restrict__ probs) {
  extern __shared__ __align__(16) char lds[];
  __shared__ LapShared<NT / 64> sh;
  const LapProblem p = probs != nullptr ? probs[blockIdx.x] : one;
  if (p.n < 1) return;
  int* freel = reinterpret_cast<int*>(p.ws + lap_array_bytes(p.n));
  const LapArrays a = lap_carve(IN_LDS ? lds : p.ws, p.n, freel);
  const int r = lap_solve<NT>(p.w, p.n, (size_t)p.ld, p.sigma, p.u_ready ? p.u_init : nullptr,
                              a, sh);
  if (threadIdx.x == 0 && p.paths_out != nullptr) *p.paths_out = r;
}

bool lap_in_lds(int max_n) { return lap_array_bytes(max_n) <= kLapLdsBytes; }

}  // namespace

size_t lap_workspace_bytes(int n) {
  return (lap_array_bytes(n) + (size_t)n * 4 + 255) / 256 * 256;
}

hipError_t launch_lap(const LapProblem* one, const LapProblem* probs, int count, int max_n,
                      hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if ((one == nullptr) == (probs == nullptr)) return hipErrorInvalidValue;
  if (one != nullptr && (count != 1 || one->n > max_n)) return hipErrorInvalidValue;
  const LapProblem p1 = one != nullptr ? *one : LapProblem{};
  const bool lds = lap_in_lds(max_n);
  const size_t shm = lds ? lap_array_bytes(max_n) : 0;
  if (max_n <= 1024) {
    if (lds)
      lap_kernel<256, true><<<count, 256, shm, s>>>(p1, probs);
    else
      lap_kernel<256, false><<<count, 256, 0, s>>>(p1, probs);
  } else if (lds) {
    const hipError_t e =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&lap_kernel<1024, true>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    lap_kernel<1024, true><<<count, 1024, shm, s>>>(p1, probs);
  } else {
    lap_kernel<1024, false><<<count, 1024, 0, s>>>(p1, probs);
  }
  return hipGetLastError();
}

}  // namespace fram
