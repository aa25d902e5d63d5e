// Memory-bound helper kernels of the FRAM path:
//   prescale   (Algorithm 1, steps 2-3): max-reduce, scale and cast to the GEMM type;
//   update     (Algorithm 1, steps 7-8): N <- (1-alpha) N + alpha D with FP64 sums for delta;
//   discretise (Algorithm 1, step 10 / eq. 2): row argmax of N;
//   objective  (eq. 1 without node term): sum_{k,l} A_kl B_{s(k) s(l)} in FP64;
// plus input validation (Sec. 3: A nonnegative and symmetric), fills and copies.
// Every reduction is two-stage with a fixed order, so results are bitwise
// reproducible run to run.
#include "fram_internal.h"

namespace fram {
namespace {

constexpr int kT = 256;

__device__ double block_sum_256(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
#pragma unroll
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ double block_max_256(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
#pragma unroll
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] = fmax(sh[tid], sh[tid + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

template <Elem E>
struct Conv;
template <>
struct Conv<Elem::F32> {
  typedef float T;
  __device__ static T from(double v) { return (float)v; }
};
template <>
struct Conv<Elem::BF16> {
  typedef __bf16 T;
  __device__ static T from(double v) { return (__bf16)(float)v; }
};
template <>
struct Conv<Elem::F16> {
  typedef _Float16 T;
  __device__ static T from(double v) { return (_Float16)(float)v; }
};

// ------------------------------------------------------------------ prescale
__global__ __launch_bounds__(kT) void max_partial_kernel(const double* __restrict__ A,
                                                         const double* __restrict__ B, size_t nn,
                                                         double* part) {
  __shared__ double sh[kT];
  double ma = -INFINITY, mb = -INFINITY;
  for (size_t t = (size_t)blockIdx.x * kT + threadIdx.x; t < nn; t += (size_t)gridDim.x * kT) {
    ma = fmax(ma, A[t]);
    mb = fmax(mb, B[t]);
  }
  ma = block_max_256(ma, sh);
  mb = block_max_256(mb, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ma;
    part[2 * blockIdx.x + 1] = mb;
  }
}

__global__ __launch_bounds__(kT) void max_final_kernel(const double* part, int nblocks,
                                                       DevState* st) {
  __shared__ double sh[kT];
  double ma = -INFINITY, mb = -INFINITY;
  for (int b = threadIdx.x; b < nblocks; b += kT) {
    ma = fmax(ma, part[2 * b]);
    mb = fmax(mb, part[2 * b + 1]);
  }
  ma = block_max_256(ma, sh);
  mb = block_max_256(mb, sh);
  if (threadIdx.x == 0) {
    st->maxA = ma;
    st->maxB = mb;
  }
}

template <Elem E>
__global__ __launch_bounds__(kT) void cast_scaled_kernel(const double* __restrict__ src, int n,
                                                         typename Conv<E>::T* __restrict__ dst,
                                                         int np, const DevState* st, int which) {
  const double m = which == 0 ? st->maxA : st->maxB;
  const double inv_ok = (m > 0.0) ? 1.0 : 0.0;
  const double den = (m > 0.0) ? m : 1.0;
  const size_t total = (size_t)np * np;
  for (size_t t = (size_t)blockIdx.x * kT + threadIdx.x; t < total; t += (size_t)gridDim.x * kT) {
    const int i = (int)(t / np), j = (int)(t % np);
    double v = 0.0;
    if (i < n && j < n) v = inv_ok * (src[(size_t)i * n + j] / den);
    dst[t] = Conv<E>::from(v);
  }
}

// ---------------------------------------------------------------- node term
__global__ __launch_bounds__(kT) void absmax_partial_kernel(const double* __restrict__ K,
                                                            size_t nn, double* part) {
  __shared__ double sh[kT];
  double m = 0.0;
  for (size_t t = (size_t)blockIdx.x * kT + threadIdx.x; t < nn; t += (size_t)gridDim.x * kT)
    m = fmax(m, fabs(K[t]));
  m = block_max_256(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ __launch_bounds__(kT) void absmax_final_kernel(const double* part, int nblocks,
                                                          DevState* st) {
  __shared__ double sh[kT];
  double m = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kT) m = fmax(m, part[b]);
  m = block_max_256(m, sh);
  if (threadIdx.x == 0) st->maxK = m;
}

// X's node term on the scale of the edge term A N B / (maxA maxB): any
// positive common factor of both terms leaves SDSN's result unchanged
// (Alg. 2 divides by max X), so this equals the paper's c-scaling.
__global__ __launch_bounds__(kT) void node_term_kernel(const double* __restrict__ K, int n,
                                                       double w, float* __restrict__ dst, int np,
                                                       const DevState* st) {
  const double a = st->maxA, b = st->maxB, mk = st->maxK;
  const double sc = (a > 0.0 && b > 0.0) ? w / (a * b) : (mk > 0.0 ? w / mk : 0.0);
  const size_t total = (size_t)np * np;
  for (size_t t = (size_t)blockIdx.x * kT + threadIdx.x; t < total; t += (size_t)gridDim.x * kT) {
    const int i = (int)(t / np), j = (int)(t % np);
    dst[t] = (i < n && j < n) ? (float)(sc * K[(size_t)i * n + j]) : 0.0f;
  }
}

__global__ __launch_bounds__(kT) void node_objective_kernel(const double* __restrict__ K,
                                                            const int32_t* __restrict__ sigma,
                                                            int n, double w, DevState* st) {
  __shared__ double sh[kT];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += kT) {
    const int j = sigma[k];
    acc += (j >= 0 && j < n) ? K[(size_t)k * n + j] : __builtin_nan("");
  }
  acc = block_sum_256(acc, sh);
  if (threadIdx.x == 0) st->objective += 2.0 * w * acc;
}

template <Elem E>
__global__ __launch_bounds__(kT) void cast_f32_kernel(const float* __restrict__ src, int n,
                                                      typename Conv<E>::T* __restrict__ dst,
                                                      int np) {
  const size_t total = (size_t)np * np;
  for (size_t t = (size_t)blockIdx.x * kT + threadIdx.x; t < total; t += (size_t)gridDim.x * kT) {
    const int i = (int)(t / np), j = (int)(t % np);
    double v = 0.0;
    if (i < n && j < n) v = (double)src[(size_t)i * n + j];
    dst[t] = Conv<E>::from(v);
  }
}

// ------------------------------------------------------------------ update
// Block b of nblocks: a grid-stride share of the rows, and its FP64 partial
// sums of delta's numerator and denominator in part[2b], part[2b + 1].
template <Elem E>
__device__ __forceinline__ void update_body(const float* __restrict__ D, float* __restrict__ N,
                                            void* Nlp, int n, int np, float alpha, double* part,
                                            int b, int nblocks) {
  __shared__ double sh[kT];
  const float c1 = 1.0f - alpha;
  double num = 0.0, den = 0.0;
  const int q = np / 4;  // float4 per row
  const size_t total = (size_t)n * q;
  for (size_t t = (size_t)b * kT + threadIdx.x; t < total; t += (size_t)nblocks * kT) {
    const size_t i = t / q, c = t % q;
    const size_t idx = i * np + 4 * c;
    const float4 o = *reinterpret_cast<const float4*>(N + idx);
    const float4 d = *reinterpret_cast<const float4*>(D + idx);
    float4 nn;
    nn.x = fmaf(alpha, d.x, c1 * o.x);
    nn.y = fmaf(alpha, d.y, c1 * o.y);
    nn.z = fmaf(alpha, d.z, c1 * o.z);
    nn.w = fmaf(alpha, d.w, c1 * o.w);
    *reinterpret_cast<float4*>(N + idx) = nn;
    if (E != Elem::F32) {
      typedef typename Conv<E>::T T;
      T* out = reinterpret_cast<T*>(Nlp) + idx;
      out[0] = Conv<E>::from(nn.x);
      out[1] = Conv<E>::from(nn.y);
      out[2] = Conv<E>::from(nn.z);
      out[3] = Conv<E>::from(nn.w);
    }
    const double ex = (double)nn.x - (double)o.x, ey = (double)nn.y - (double)o.y;
    const double ez = (double)nn.z - (double)o.z, ew = (double)nn.w - (double)o.w;
    num += (ex * ex + ey * ey) + (ez * ez + ew * ew);
    den += ((double)nn.x * nn.x + (double)nn.y * nn.y) + ((double)nn.z * nn.z + (double)nn.w * nn.w);
  }
  num = block_sum_256(num, sh);
  den = block_sum_256(den, sh);
  if (threadIdx.x == 0) {
    part[2 * b] = num;
    part[2 * b + 1] = den;
  }
}

template <Elem E>
__global__ __launch_bounds__(kT) void update_kernel(const float* __restrict__ D,
                                                    float* __restrict__ N, void* Nlp, int n,
                                                    int np, float alpha, double* part) {
  update_body<E>(D, N, Nlp, n, np, alpha, part, blockIdx.x, gridDim.x);
}

// The updates of many pairs (job blockIdx.y), each with its own block count.
template <Elem E>
__global__ __launch_bounds__(kT) void update_group_kernel(const UpdateJob* __restrict__ jobs,
                                                          float alpha) {
  const UpdateJob j = jobs[blockIdx.y];
  if ((int)blockIdx.x >= j.nblocks) return;
  update_body<E>(j.D, j.N, j.Nlp, j.n, j.np, alpha, j.part, blockIdx.x, j.nblocks);
}

__device__ __forceinline__ void delta_final_body(const double* part, int nblocks, DevState* st) {
  __shared__ double sh[kT];
  double num = 0.0, den = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kT) {
    num += part[2 * b];
    den += part[2 * b + 1];
  }
  num = block_sum_256(num, sh);
  den = block_sum_256(den, sh);
  if (threadIdx.x == 0) {
    st->dnum = num;
    st->dden = den;
    st->delta = den > 0.0 ? sqrt(num) / sqrt(den) : 0.0;
  }
}

__global__ __launch_bounds__(kT) void delta_final_kernel(const double* part, int nblocks,
                                                         DevState* st) {
  delta_final_body(part, nblocks, st);
}

__global__ __launch_bounds__(kT) void delta_group_kernel(const UpdateJob* __restrict__ jobs) {
  const UpdateJob j = jobs[blockIdx.x];
  delta_final_body(j.part, j.nblocks, j.st);
}

// ------------------------------------------------------------------ validation
// Input checks of a graph matrix (finite, non-negative, symmetric) by tile
// pairs: workgroup (J, I) with I <= J reads tile (I, J) into LDS and tile
// (J, I) row by row, so both reads are coalesced and each element is
// compared with its mirror image through LDS.  Every element is checked for
// finiteness and sign once, every pair (i, j) for symmetry once (a NaN fails
// both, as NaN != NaN).  Workgroups below the diagonal leave at once.
constexpr int kVT = 32;  // tile edge (kT = 256 threads: 32 x 8, four rows each)
__global__ __launch_bounds__(kT) void validate_kernel(const double* __restrict__ A, int n,
                                                      DevState* st) {
  __shared__ double t[kVT][kVT + 1];
  __shared__ int sflag;
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi > bj) return;
  if (threadIdx.x == 0) sflag = 0;
  const int tx = threadIdx.x % kVT, ty = threadIdx.x / kVT;
  int f = 0;
#pragma unroll
  for (int k = 0; k < kVT / 8; ++k) {
    const int r = bi * kVT + ty + 8 * k, c = bj * kVT + tx;
    double v = 0.0;
    if (r < n && c < n) {
      v = A[(size_t)r * n + c];
      if (!isfinite(v)) f |= 1;
      if (v < 0.0) f |= 2;
    }
    t[ty + 8 * k][tx] = v;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kVT / 8; ++k) {
    // Element (r, c) of tile (J, I) mirrors (c, r) of tile (I, J).
    const int r = bj * kVT + ty + 8 * k, c = bi * kVT + tx;
    if (r >= n || c >= n) continue;
    const double m = t[tx][ty + 8 * k];
    if (bi != bj) {
      const double v = A[(size_t)r * n + c];
      if (!isfinite(v)) f |= 1;
      if (v < 0.0) f |= 2;
      if (v != m) f |= 4;
    } else if (t[ty + 8 * k][tx] != m) {
      f |= 4;
    }
  }
  if (f) atomicOr(&sflag, f);
  __syncthreads();
  if (threadIdx.x == 0 && sflag) atomicOr(&st->invalid, sflag);
}

// ------------------------------------------------------------------ discretise
__global__ __launch_bounds__(kT) void row_argmax_kernel(const float* __restrict__ N, int n,
                                                        int np, int32_t* __restrict__ sigma,
                                                        double* __restrict__ u) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
  if (row >= n) return;
  const float* r = N + (size_t)row * np;
  float best = -INFINITY;
  int bi = n;  // sentinel larger than any index
  for (int j = lane; j < n; j += 64) {
    const float v = r[j];
    if (v > best) {
      best = v;
      bi = j;
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float ob = __shfl_xor(best, off);
    const int oi = __shfl_xor(bi, off);
    if (ob > best || (ob == best && oi < bi)) {
      best = ob;
      bi = oi;
    }
  }
  if (lane == 0) {
    sigma[row] = bi < n ? bi : 0;
    if (u != nullptr) u[row] = -(double)best;
  }
}

// ------------------------------------------------------------------ objective
__global__ __launch_bounds__(kT) void objective_kernel(const double* __restrict__ A,
                                                       const double* __restrict__ B,
                                                       const int32_t* __restrict__ sigma, int n,
                                                       double* part) {
  __shared__ double sh[kT];
  double acc = 0.0;
  // An index outside [0, n) (a failed assignment) makes the sum NaN instead
  // of being read.
  for (int k = blockIdx.x; k < n; k += gridDim.x) {
    const int sk = sigma[k];
    if (sk < 0 || sk >= n) {
      acc = __builtin_nan("");
      continue;
    }
    const double* ar = A + (size_t)k * n;
    const double* br = B + (size_t)sk * n;
    for (int l = threadIdx.x; l < n; l += kT) {
      const int sl = sigma[l];
      acc += (sl >= 0 && sl < n) ? ar[l] * br[sl] : __builtin_nan("");
    }
  }
  acc = block_sum_256(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(kT) void objective_final_kernel(const double* part, int nblocks,
                                                             DevState* st) {
  __shared__ double sh[kT];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kT) acc += part[b];
  acc = block_sum_256(acc, sh);
  if (threadIdx.x == 0) st->objective = acc;
}

// ------------------------------------------------------------------ fills
__global__ __launch_bounds__(kT) void zero_kernel(uint4* p, size_t n16, unsigned char* tail,
                                                  size_t ntail) {
  for (size_t t = (size_t)blockIdx.x * kT + threadIdx.x; t < n16; t += (size_t)gridDim.x * kT)
    p[t] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kT) void copy_f32_kernel(const float* __restrict__ src, int ld_src,
                                                      float* __restrict__ dst, int ld_dst, int n) {
  const size_t total = (size_t)n * n;
  for (size_t t = (size_t)blockIdx.x * kT + threadIdx.x; t < total; t += (size_t)gridDim.x * kT) {
    const size_t i = t / n, j = t % n;
    dst[i * ld_dst + j] = src[i * ld_src + j];
  }
}

// ------------------------------------------------------------ DSPFP criterion
__global__ __launch_bounds__(kT) void nmax_partial_kernel(const float* __restrict__ N, int n,
                                                          int np, double* part) {
  __shared__ double sh[kT];
  double m = -__builtin_inf();
  const size_t total = (size_t)n * n;
  for (size_t t = (size_t)blockIdx.x * kT + threadIdx.x; t < total; t += (size_t)gridDim.x * kT)
    m = fmax(m, (double)N[(t / n) * np + t % n]);
  m = block_max_256(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ __launch_bounds__(kT) void nmax_final_kernel(const double* part, int nblocks,
                                                        DevState* st) {
  __shared__ double sh[kT];
  double m = -__builtin_inf();
  for (int b = threadIdx.x; b < nblocks; b += kT) m = fmax(m, part[b]);
  m = block_max_256(m, sh);
  if (threadIdx.x == 0) {
    st->nmax_prev = st->nmax;
    st->nmax = m;
  }
}

__global__ __launch_bounds__(kT) void crit_partial_kernel(const float* __restrict__ N,
                                                          const float* __restrict__ P, int n,
                                                          int np, const DevState* st,
                                                          double* part) {
  __shared__ double sh[kT];
  const double a = st->nmax, b = st->nmax_prev;
  double m = 0.0;
  if (a > 0.0 && b > 0.0) {
    const size_t total = (size_t)n * n;
    for (size_t t = (size_t)blockIdx.x * kT + threadIdx.x; t < total;
         t += (size_t)gridDim.x * kT) {
      const size_t idx = (t / n) * np + t % n;
      m = fmax(m, fabs((double)N[idx] / a - (double)P[idx] / b));
    }
  }
  m = block_max_256(m, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

__global__ __launch_bounds__(kT) void crit_final_kernel(const double* part, int nblocks,
                                                        DevState* st) {
  __shared__ double sh[kT];
  double m = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kT) m = fmax(m, part[b]);
  m = block_max_256(m, sh);
  if (threadIdx.x == 0)
    st->delta = (st->nmax > 0.0 && st->nmax_prev > 0.0) ? m : __builtin_inf();
}

int grid_for(size_t work) {
  size_t b = (work + kT - 1) / kT;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

int max_blocks(int n) { return grid_for((size_t)n * n); }
int update_blocks(int n) { return grid_for((size_t)n * n / 4 + 1); }
int objective_blocks(int n) { return n < 1024 ? n : 1024; }

hipError_t launch_maxes(const double* A, const double* B, int n, double* part, int nblocks,
                        DevState* st, hipStream_t s) {
  max_partial_kernel<<<nblocks, kT, 0, s>>>(A, B, (size_t)n * n, part);
  max_final_kernel<<<1, kT, 0, s>>>(part, nblocks, st);
  return hipGetLastError();
}

hipError_t launch_cast_scaled(Elem e, const double* src, int n, void* dst, int np,
                              const DevState* st, int which, hipStream_t s) {
  const int g = grid_for((size_t)np * np);
  switch (e) {
    case Elem::F32:
      cast_scaled_kernel<Elem::F32><<<g, kT, 0, s>>>(src, n, (float*)dst, np, st, which);
      break;
    case Elem::BF16:
      cast_scaled_kernel<Elem::BF16><<<g, kT, 0, s>>>(src, n, (__bf16*)dst, np, st, which);
      break;
    case Elem::F16:
      cast_scaled_kernel<Elem::F16><<<g, kT, 0, s>>>(src, n, (_Float16*)dst, np, st, which);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_cast_f32(Elem e, const float* src, int n, void* dst, int np, hipStream_t s) {
  const int g = grid_for((size_t)np * np);
  switch (e) {
    case Elem::F32:
      cast_f32_kernel<Elem::F32><<<g, kT, 0, s>>>(src, n, (float*)dst, np);
      break;
    case Elem::BF16:
      cast_f32_kernel<Elem::BF16><<<g, kT, 0, s>>>(src, n, (__bf16*)dst, np);
      break;
    case Elem::F16:
      cast_f32_kernel<Elem::F16><<<g, kT, 0, s>>>(src, n, (_Float16*)dst, np);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_update(Elem e, const float* D, float* N, void* Nlp, int n, int np,
                         double alpha, double* part, int nblocks, DevState* st,
                         hipStream_t s) {
  if (np % 4 != 0) return hipErrorInvalidValue;
  switch (e) {
    case Elem::F32:
      update_kernel<Elem::F32><<<nblocks, kT, 0, s>>>(D, N, Nlp, n, np, (float)alpha, part);
      break;
    case Elem::BF16:
      update_kernel<Elem::BF16><<<nblocks, kT, 0, s>>>(D, N, Nlp, n, np, (float)alpha, part);
      break;
    case Elem::F16:
      update_kernel<Elem::F16><<<nblocks, kT, 0, s>>>(D, N, Nlp, n, np, (float)alpha, part);
      break;
  }
  delta_final_kernel<<<1, kT, 0, s>>>(part, nblocks, st);
  return hipGetLastError();
}

hipError_t launch_update_group(Elem e, const UpdateJob* jobs, int count, int max_blocks,
                               double alpha, hipStream_t s) {
  if (count < 1) return hipSuccess;
  if (count > 65535 || max_blocks < 1) return hipErrorInvalidValue;
  const dim3 grid(max_blocks, count);
  switch (e) {
    case Elem::F32:
      update_group_kernel<Elem::F32><<<grid, kT, 0, s>>>(jobs, (float)alpha);
      break;
    case Elem::BF16:
      update_group_kernel<Elem::BF16><<<grid, kT, 0, s>>>(jobs, (float)alpha);
      break;
    case Elem::F16:
      update_group_kernel<Elem::F16><<<grid, kT, 0, s>>>(jobs, (float)alpha);
      break;
  }
  delta_group_kernel<<<count, kT, 0, s>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_delta_final(const double* part, int nblocks, DevState* st, hipStream_t s) {
  delta_final_kernel<<<1, kT, 0, s>>>(part, nblocks, st);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n16 = bytes / 16;
  const size_t ntail = bytes % 16;
  zero_kernel<<<grid_for(n16 + 1), kT, 0, s>>>(static_cast<uint4*>(p), n16,
                                                static_cast<unsigned char*>(p) + n16 * 16, ntail);
  return hipGetLastError();
}

hipError_t launch_validate(const double* A, int n, DevState* st, hipStream_t s) {
  if (n < 1) return hipSuccess;
  const int nt = (n + kVT - 1) / kVT;
  validate_kernel<<<dim3(nt, nt), kT, 0, s>>>(A, n, st);
  return hipGetLastError();
}

hipError_t launch_row_argmax(const float* N, int n, int np, int32_t* sigma, hipStream_t s,
                             double* u) {
  const int rows_per_block = kT / 64;
  row_argmax_kernel<<<(n + rows_per_block - 1) / rows_per_block, kT, 0, s>>>(N, n, np, sigma, u);
  return hipGetLastError();
}

hipError_t launch_objective(const double* A, const double* B, const int32_t* sigma, int n,
                            double* part, int nblocks, DevState* st, hipStream_t s) {
  objective_kernel<<<nblocks, kT, 0, s>>>(A, B, sigma, n, part);
  objective_final_kernel<<<1, kT, 0, s>>>(part, nblocks, st);
  return hipGetLastError();
}

hipError_t launch_node_term(const double* K, int n, double w, float* dst, int np, double* part,
                            int nblocks, DevState* st, hipStream_t s) {
  absmax_partial_kernel<<<nblocks, kT, 0, s>>>(K, (size_t)n * n, part);
  absmax_final_kernel<<<1, kT, 0, s>>>(part, nblocks, st);
  node_term_kernel<<<grid_for((size_t)np * np), kT, 0, s>>>(K, n, w, dst, np, st);
  return hipGetLastError();
}

hipError_t launch_node_objective(const double* K, const int32_t* sigma, int n, double w,
                                 DevState* st, hipStream_t s) {
  node_objective_kernel<<<1, kT, 0, s>>>(K, sigma, n, w, st);
  return hipGetLastError();
}

hipError_t launch_dspfp_criterion(const float* N, const float* P, int n, int np, double* part,
                                  int nblocks, DevState* st, hipStream_t s) {
  nmax_partial_kernel<<<nblocks, kT, 0, s>>>(N, n, np, part);
  nmax_final_kernel<<<1, kT, 0, s>>>(part, nblocks, st);
  crit_partial_kernel<<<nblocks, kT, 0, s>>>(N, P, n, np, st, part);
  crit_final_kernel<<<1, kT, 0, s>>>(part, nblocks, st);
  return hipGetLastError();
}

hipError_t launch_copy_f32(const float* src, int ld_src, float* dst, int ld_dst, int n,
                           hipStream_t s) {
  copy_f32_kernel<<<grid_for((size_t)n * n), kT, 0, s>>>(src, ld_src, dst, ld_dst, n);
  return hipGetLastError();
}

}  // namespace fram
