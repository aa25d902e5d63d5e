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

// The state of the parallel bidding rounds (LapBidState), after the partial
// column minima.
__host__ __device__ inline size_t bid_offset(int n) {
  return (vpart_offset(n) + (size_t)col_chunks(n) * n * 8 + 255) / 256 * 256;
}
__host__ __device__ inline size_t bid_bytes(int n) {
  return ((size_t)n * (8 + 8 + 4 + 4 + 4 + 4 + 8 + 4 + 8 + 8) + 64 + 255) / 256 * 256;
}
__host__ __device__ inline LapBidState bid_carve(char* ws, int n) {
  char* b = ws + bid_offset(n);
  LapBidState s;
  s.u = reinterpret_cast<double*>(b);
  s.v = s.u + n;
  s.newu = s.v + n;
  s.drop = s.newu + n;
  s.key = reinterpret_cast<unsigned long long*>(s.drop + n);
  s.row_of = reinterpret_cast<int*>(s.key + n);
  s.col_of = s.row_of + n;
  s.list[0] = s.col_of + n;
  s.list[1] = s.list[0] + n;
  s.tgt = s.list[1] + n;
  s.ctl = s.tgt + n;
  return s;
}

// Smallest n for which the assignment bids in parallel rounds first.
constexpr int kBidMinN = 1024;
// Rounds launched (the kernels of the rounds after the stop return at once).
// On the n = 4000 workloads the rounds still match a row every few rounds
// after 64 of them, each saving a path search far longer than a round
// (measured assignment: 16.3 ms with 64 rounds, 15.6 ms with 128, 23.8 ms with
// 256 before the search read ahead, against 23.1 with 128).
constexpr int kBidRounds = 128;

// Start of the bidding rounds: u = -row maxima (given), v = the column
// minima, the tight argmax pairs matched (a column to its lowest claiming
// row), the other rows listed.  Three launches, as each step reads what the
// previous one wrote across the grid.
__global__ __launch_bounds__(256) void bid_init_kernel(LapBidState s, int n,
                                                       const double* __restrict__ u_init,
                                                       const double* __restrict__ vpart,
                                                       int chunks) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t == 0) {
    s.ctl[0] = s.ctl[1] = s.ctl[2] = s.ctl[4] = s.ctl[6] = s.ctl[7] = 0;
    s.ctl[3] = n + 1;
  }
  if (t >= n) return;
  double vj = vpart[t];
  for (int c = 1; c < chunks; ++c) vj = fmin(vj, vpart[(size_t)c * n + t]);
  s.v[t] = vj;
  s.u[t] = u_init[t];
  s.row_of[t] = INT_MAX;
  s.key[t] = 0;
  s.tgt[t] = -1;
}

__global__ __launch_bounds__(256) void bid_match_kernel(LapBidState s, const float* __restrict__ W,
                                                        int n, int ld,
                                                        const int32_t* __restrict__ sigma) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int j = sigma[i];
  if (j >= 0 && j < n && (-(double)W[(size_t)i * ld + j]) - s.u[i] - s.v[j] == 0.0)
    atomicMin(&s.row_of[j], i);
}

__global__ __launch_bounds__(256) void bid_list_kernel(LapBidState s, int n,
                                                       const int32_t* __restrict__ sigma) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const int j = sigma[t];
  const bool matched = j >= 0 && j < n && s.row_of[j] == t;
  s.col_of[t] = matched ? j : -1;
  if (!matched) {
    s.list[0][atomicAdd(&s.ctl[0], 1)] = t;
    atomicAdd(&s.ctl[6], 1);  // rows the row maxima left free (reported)
  }
  // A column nobody kept: unmatched.  (Reading a row_of that another thread
  // turns from INT_MAX to -1 gives "not this row" either way.)
  if (s.row_of[t] == INT_MAX) s.row_of[t] = -1;
}

// Round r (list p = r & 1): one wave per listed row, the grid's waves
// striding over the list (a grid sized for the first round's list would
// mostly start empty blocks in the later, short rounds).  The last workgroup
// to finish its bids then resolves them -- each column to its largest bid,
// displaced owners listed for the next round -- and applies the stop rule:
// no row left, or the count not fallen for kBidStall rounds.  One launch per
// round.  The bids are written and read at the device-coherent level (agent
// scope), and every wave waits for its own writes to complete before its
// workgroup counts itself done in ctl[7], so the last workgroup to count sees
// every bid without a cache flush (a fence per workgroup and round, which
// writes the L2 back, cost more than the launches it saves).
__global__ __launch_bounds__(256) void bid_round_kernel(LapBidState s, const float* __restrict__ W,
                                                        int n, int ld, int p) {
  __shared__ int s_last;
  if (s.ctl[2] != 0) return;
  const int q = p ^ 1;
  // The next list's count restarts from 0 (agent scope: the last workgroup's
  // appends, possibly on another XCD, count on from it).
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(&s.ctl[q], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const int count = s.ctl[p];
  for (int w = blockIdx.x * 4 + (threadIdx.x >> 6); w < count; w += gridDim.x * 4)
    lap_bid_row(W, n, (size_t)ld, s, s.list[p][w]);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    s_last = __hip_atomic_fetch_add(&s.ctl[7], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
             (int)gridDim.x - 1;
  __syncthreads();
  if (!s_last) return;
  for (int t = threadIdx.x; t < count; t += 256) lap_resolve_row(s, s.list[p][t], q);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int c = __hip_atomic_load(&s.ctl[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (c < s.ctl[3]) {
      s.ctl[3] = c;
      s.ctl[4] = 0;
    } else {
      s.ctl[4] += 1;
    }
    if (c == 0 || s.ctl[4] >= kBidStall) s.ctl[2] = 1;
    s.ctl[7] = 0;
  }
}

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

// One problem with its row reduction given, n <= NT * C: the solver with
// the column state in registers (lap_solve_reg), NT threads.  V4: rows read
// as whole float4 groups (n % 4 == 0, n >= 4, 16-byte aligned rows).
template <int NT, int C, bool V4>
__global__ __launch_bounds__(NT) void lap_reg_kernel(LapProblem p, int after_bids) {
  extern __shared__ __align__(16) char lds[];
  __shared__ LapShared<NT / 64> sh;
  const LapRegArrays a = lap_reg_carve(lds, p.n);
  const double* vpart = reinterpret_cast<const double*>(p.ws + vpart_offset(p.n));
  const LapBidState bs = bid_carve(p.ws, p.n);
  const int r = lap_solve_reg<NT, C, V4>(p.w, p.n, (size_t)p.ld, p.sigma, p.u_init, vpart,
                                         col_chunks(p.n), a, sh, after_bids ? &bs : nullptr);
  if (threadIdx.x == 0 && p.paths_out != nullptr) *p.paths_out = r;
}

template <int NT, int C>
hipError_t launch_lap_reg(const LapProblem& p, hipStream_t s) {
  const int n = p.n;
  const bool bids = n >= kBidMinN;
  if (bids) {
    // The bidding rounds on the whole device, then the paths in one workgroup.
    const LapBidState bs = bid_carve(p.ws, n);
    const double* vpart = reinterpret_cast<const double*>(p.ws + vpart_offset(n));
    const int blocks = (n + 255) / 256;
    const int round_blocks = (n + 3) / 4 < 256 ? (n + 3) / 4 : 256;
    bid_init_kernel<<<blocks, 256, 0, s>>>(bs, n, p.u_init, vpart, col_chunks(n));
    bid_match_kernel<<<blocks, 256, 0, s>>>(bs, p.w, n, p.ld, p.sigma);
    bid_list_kernel<<<blocks, 256, 0, s>>>(bs, n, p.sigma);
    for (int r = 0; r < kBidRounds; ++r) {
      const int q = r & 1;
      bid_round_kernel<<<round_blocks, 256, 0, s>>>(bs, p.w, n, p.ld, q);
    }
  }
  const size_t shm = lap_reg_lds_bytes(n);
  const bool v4 = n >= 4 && n % 4 == 0 && p.ld % 4 == 0 &&
                  (reinterpret_cast<uintptr_t>(p.w) & 15) == 0;
  const void* fn = v4 ? reinterpret_cast<const void*>(&lap_reg_kernel<NT, C, true>)
                      : reinterpret_cast<const void*>(&lap_reg_kernel<NT, C, false>);
  const hipError_t e =
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e != hipSuccess) return e;
  if (v4)
    lap_reg_kernel<NT, C, true><<<1, NT, shm, s>>>(p, bids ? 1 : 0);
  else
    lap_reg_kernel<NT, C, false><<<1, NT, shm, s>>>(p, bids ? 1 : 0);
  return hipGetLastError();
}

bool lap_in_lds(int max_n) { return lap_array_bytes(max_n) <= kLapLdsBytes; }

}  // namespace

size_t lap_workspace_bytes(int n) {
  return bid_offset(n) + bid_bytes(n);
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
    if (p1.n <= 256 * 4) return launch_lap_reg<256, 4>(p1, s);
    if (p1.n <= 256 * 8) return launch_lap_reg<256, 8>(p1, s);
    if (p1.n <= 256 * 16) return launch_lap_reg<256, 16>(p1, s);
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
