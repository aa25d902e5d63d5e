// Launcher of the device linear assignment (lap_device.h): one workgroup per
// problem.  Its arrays live in LDS when they fit (n <= 4400), else in the
// problem's global workspace; the unmatched-row list is always in the
// workspace, after the arrays.
#include "lap_device.h"

namespace fram {
namespace {

constexpr size_t kLapLdsBytes = 160 * 1024 - 1024;  // minus the static LDS
constexpr int kColChunks = 32;  // row chunks of the column-minimum pass

// Offset in ws of the partial column minima (after the arrays and the
// unmatched-row list).
__host__ __device__ inline size_t vpart_offset(int n) {
  return (lap_array_bytes(n) + (size_t)n * 4 + 15) / 16 * 16;
}

__host__ __device__ inline int col_chunks(int n) { return n < kColChunks ? n : kColChunks; }

// Partial column minima of the reduced costs after the row reduction:
// part[c * n + j] = min over the rows i of chunk c of (-(double)w_ij - u_i),
// finite values only (a column with none gets 0, i.e. no reduction).
__global__ __launch_bounds__(256) void colmin_kernel(const float* __restrict__ w, int n, int ld,
                                                     const double* __restrict__ u,
                                                     double* __restrict__ part, int chunks) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const int c = blockIdx.y;
  const int per = (n + chunks - 1) / chunks;
  const int i0 = c * per, i1 = (i0 + per < n) ? i0 + per : n;
  double m = __builtin_inf();
  for (int i = i0; i < i1; ++i) {
    const double h = -(double)w[(size_t)i * ld + j] - u[i];
    if (isfinite(h) && h < m) m = h;
  }
  part[(size_t)c * n + j] = isfinite(m) ? m : 0.0;
}

template <int NT, bool IN_LDS>
__global__ __launch_bounds__(NT) void lap_kernel(LapProblem one,
                                                 const LapProblem* __restrict__ probs) {
  extern __shared__ __align__(16) char lds[];
  __shared__ LapShared<NT / 64> sh;
  const LapProblem p = probs != nullptr ? probs[blockIdx.x] : one;
  if (p.n < 1) return;
  int* freel = reinterpret_cast<int*>(p.ws + lap_array_bytes(p.n));
  const LapArrays a = lap_carve(IN_LDS ? lds : p.ws, p.n, freel);
  const bool ready = p.u_ready != 0;
  // Column minima exist only for the single problem (see launch_lap).
  const double* vpart = (ready && probs == nullptr)
                            ? reinterpret_cast<const double*>(p.ws + vpart_offset(p.n))
                            : nullptr;
  const int r = lap_solve<NT>(p.w, p.n, (size_t)p.ld, p.sigma, ready ? p.u_init : nullptr, vpart,
                              col_chunks(p.n), a, sh);
  if (threadIdx.x == 0 && p.paths_out != nullptr) *p.paths_out = r;
}

// One problem with its row reduction given, n <= 256 * C: the solver with
// the column state in registers (lap_solve_reg), 256 threads.
template <int C>
__global__ __launch_bounds__(256) void lap_reg_kernel(LapProblem p) {
  extern __shared__ __align__(16) char lds[];
  __shared__ LapShared<4> sh;
  const LapRegArrays a = lap_reg_carve(lds, p.n);
  const double* vpart = reinterpret_cast<const double*>(p.ws + vpart_offset(p.n));
  const int r = lap_solve_reg<256, C>(p.w, p.n, (size_t)p.ld, p.sigma, p.u_init, vpart,
                                      col_chunks(p.n), a, sh);
  if (threadIdx.x == 0 && p.paths_out != nullptr) *p.paths_out = r;
}

template <int C>
hipError_t launch_lap_reg(const LapProblem& p, hipStream_t s) {
  const size_t shm = lap_reg_lds_bytes(p.n);
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&lap_reg_kernel<C>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  lap_reg_kernel<C><<<1, 256, shm, s>>>(p);
  return hipGetLastError();
}

bool lap_in_lds(int max_n) { return lap_array_bytes(max_n) <= kLapLdsBytes; }

}  // namespace

size_t lap_workspace_bytes(int n) {
  return (vpart_offset(n) + (size_t)col_chunks(n) * n * 8 + 255) / 256 * 256;
}

hipError_t launch_lap(const LapProblem* one, const LapProblem* probs, int count, int max_n,
                      hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if ((one == nullptr) == (probs == nullptr)) return hipErrorInvalidValue;
  if (one != nullptr && (count != 1 || one->n > max_n)) return hipErrorInvalidValue;
  const LapProblem p1 = one != nullptr ? *one : LapProblem{};
  // Column reduction for problems whose row reduction is given: one pass over
  // the matrix by the whole device before the single-workgroup solve.  A
  // problem array (batched problems) starts from v = 0.
  if (one != nullptr && p1.u_ready && p1.n > 0) {
    const int chunks = col_chunks(p1.n);
    const dim3 grid((p1.n + 255) / 256, chunks);
    colmin_kernel<<<grid, 256, 0, s>>>(p1.w, p1.n, p1.ld, p1.u_init,
                                       reinterpret_cast<double*>(p1.ws + vpart_offset(p1.n)),
                                       chunks);
  }
  // A single problem with its row reduction given and n <= 4096: the
  // register-resident solver.
  if (one != nullptr && p1.u_ready && p1.n > 0) {
    if (p1.n <= 256 * 4) return launch_lap_reg<4>(p1, s);
    if (p1.n <= 256 * 8) return launch_lap_reg<8>(p1, s);
    if (p1.n <= 256 * 16) return launch_lap_reg<16>(p1, s);
  }
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
