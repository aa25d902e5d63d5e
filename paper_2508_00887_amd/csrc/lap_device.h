// Exact linear assignment by one workgroup, for the discretisation of
// Algorithm 1, step 10: M = argmin_{P in Pi} ||P - N||_F, i.e. the
// permutation sigma maximising sum_i N[i, sigma(i)] (eq. 2), which the paper
// obtains with the Hungarian method (Sec. 6, complexity paragraph).
//
// Method: shortest augmenting paths with row and column potentials (the
// Hungarian method in its Dijkstra form).  With costs c_ij = -N_ij, dual
// variables u_i, v_j keep every reduced cost c_ij - u_i - v_j >= 0 and make
// every matched pair tight.  The start is the dual-feasible partial matching
// of the row maxima (u_i = min_j c_ij; v_j = min_i (c_ij - u_i) when the
// column minima are supplied, else 0): a row keeps its argmax column unless a
// lower-numbered row took it first.  Two passes of augmenting row reduction
// (Jonker and Volgenant, 1987) then let the unmatched rows bid: a row takes
// the column of least reduced cost c_ij - v_j, lowers that column's price
// until its second choice is as good, and displaces the column's owner, which
// bids next (bounded in total, so a bidding war cannot run on).  Each row
// still unmatched, in list order, finally grows a shortest-path tree over the
// columns until it reaches an unmatched column, updates the potentials and
// flips the path.  When the row maxima already form a permutation there is
// nothing to augment.
//
// Columns are dealt to threads round-robin and each thread owns the
// distance, predecessor and scanned flag of its columns, so one step of the
// tree growth needs one barrier: every wave posts its (distance, column)
// minimum, and after the barrier every thread reduces the same posted values
// to the same winner.  Ties go to the lowest column and all arithmetic is
// FP64 in a fixed order, so the result does not depend on the thread count.
#pragma once

#include <limits.h>

#include "fram_internal.h"

namespace fram {

// Bytes of the per-problem arrays u, v, dist (FP64), row_of, col_of, pred
// (int32), scanned (u8), rounded up to 16.  The unmatched-row list (int32[n])
// is placed by the caller.
__host__ __device__ inline size_t lap_array_bytes(int n) {
  return ((size_t)n * (3 * 8 + 3 * 4 + 1) + 15) / 16 * 16;
}

struct LapArrays {
  double* u;
  double* v;
  double* dist;
  int* row_of;
  int* col_of;
  int* pred;
  unsigned char* scanned;
  int* freel;
};

__device__ inline LapArrays lap_carve(char* base, int n, int* freel) {
  LapArrays a;
  a.u = reinterpret_cast<double*>(base);
  a.v = a.u + n;
  a.dist = a.v + n;
  a.row_of = reinterpret_cast<int*>(a.dist + n);
  a.col_of = a.row_of + n;
  a.pred = a.col_of + n;
  a.scanned = reinterpret_cast<unsigned char*>(a.pred + n);
  a.freel = freel;
  return a;
}

template <int NW>
struct LapShared {
  double wd[2][NW];
  int wj[2][NW];
  double w2d[2][NW];  // per wave: the best column outside the wave's best thread
  int w2j[2][NW];
  int cnt[NW];
  double b1[NW], b2[NW];  // per-wave best and second-best reduced cost of a bid
  int c1[NW], c2[NW];     // ... and their columns
};

// (value, column) pairs in lexicographic order: the lower column wins ties.
__device__ __forceinline__ bool lap_lex_less(double a, int ja, double b, int jb) {
  return a < b || (a == b && ja < jb);
}

// Best two of the union of two sorted pairs (x1 before x2) and (y1 before y2),
// written as selects so that the values stay in registers.
__device__ __forceinline__ void lap_top2_merge(double& x1, int& i1, double& x2, int& i2,
                                               double y1, int k1, double y2, int k2) {
  const bool yf = lap_lex_less(y1, k1, x1, i1);  // y1 becomes the best
  // Second best: the better of (x1, y2) if y1 leads, else of (x2, y1).
  const double ca = yf ? x1 : x2, cb = yf ? y2 : y1;
  const int ia = yf ? i1 : i2, ib = yf ? k2 : k1;
  const bool bf = lap_lex_less(cb, ib, ca, ia);
  x1 = yf ? y1 : x1;
  i1 = yf ? k1 : i1;
  x2 = bf ? cb : ca;
  i2 = bf ? ib : ia;
}

// Lane exchanges inside a 16-lane DPP row (no LDS round trip).
template <int CTRL>
__device__ __forceinline__ int lap_dpp(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double lap_dpp(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = lap_dpp<CTRL>((int)b), hi = lap_dpp<CTRL>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double lap_readlane(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ void lap_better(double& d, int& j, double od, int oj) {
  if (od < d || (od == d && oj < j)) {
    d = od;
    j = oj;
  }
}

// Lexicographic minimum of (d, j) over the 64 lanes of a wave, in every
// lane: a butterfly inside each DPP row (neighbour, pair, half-row mirror,
// row mirror), then the four row results.  The minimum of a total order does
// not depend on the order of combination.  All 64 lanes must take part.
__device__ __forceinline__ void lap_wave_min(double& d, int& j) {
  lap_better(d, j, lap_dpp<0xB1>(d), lap_dpp<0xB1>(j));
  lap_better(d, j, lap_dpp<0x4E>(d), lap_dpp<0x4E>(j));
  lap_better(d, j, lap_dpp<0x141>(d), lap_dpp<0x141>(j));
  lap_better(d, j, lap_dpp<0x140>(d), lap_dpp<0x140>(j));
  double r = lap_readlane(d, 0);
  int rj = __builtin_amdgcn_readlane(j, 0);
#pragma unroll
  for (int row = 16; row < 64; row += 16)
    lap_better(r, rj, lap_readlane(d, row), __builtin_amdgcn_readlane(j, row));
  d = r;
  j = rj;
}

// Best two (value, column) pairs over the 64 lanes of a wave, in every lane,
// the same way.
__device__ __forceinline__ void lap_wave_top2(double& m1, int& j1, double& m2, int& j2) {
#define LAP_TOP2_STEP(CTRL)                                                            \
  lap_top2_merge(m1, j1, m2, j2, lap_dpp<CTRL>(m1), lap_dpp<CTRL>(j1), lap_dpp<CTRL>(m2), \
                 lap_dpp<CTRL>(j2))
  LAP_TOP2_STEP(0xB1);
  LAP_TOP2_STEP(0x4E);
  LAP_TOP2_STEP(0x141);
  LAP_TOP2_STEP(0x140);
#undef LAP_TOP2_STEP
  double r1 = lap_readlane(m1, 0), r2 = lap_readlane(m2, 0);
  int k1 = __builtin_amdgcn_readlane(j1, 0), k2 = __builtin_amdgcn_readlane(j2, 0);
#pragma unroll
  for (int row = 16; row < 64; row += 16)
    lap_top2_merge(r1, k1, r2, k2, lap_readlane(m1, row), __builtin_amdgcn_readlane(j1, row),
                   lap_readlane(m2, row), __builtin_amdgcn_readlane(j2, row));
  m1 = r1;
  j1 = k1;
  m2 = r2;
  j2 = k2;
}

// Minimum over the 64 lanes of a wave, in every lane (no NaN may take part:
// then the minimum of doubles is exact, and unique up to the sign of zero).
__device__ __forceinline__ double lap_wave_fmin(double d) {
  d = fmin(d, lap_dpp<0xB1>(d));
  d = fmin(d, lap_dpp<0x4E>(d));
  d = fmin(d, lap_dpp<0x141>(d));
  d = fmin(d, lap_dpp<0x140>(d));
  return fmin(fmin(lap_readlane(d, 0), lap_readlane(d, 16)),
              fmin(lap_readlane(d, 32), lap_readlane(d, 48)));
}
__device__ __forceinline__ int lap_wave_imin(int k) {
  k = min(k, lap_dpp<0xB1>(k));
  k = min(k, lap_dpp<0x4E>(k));
  k = min(k, lap_dpp<0x141>(k));
  k = min(k, lap_dpp<0x140>(k));
  return min(min(__builtin_amdgcn_readlane(k, 0), __builtin_amdgcn_readlane(k, 16)),
             min(__builtin_amdgcn_readlane(k, 32), __builtin_amdgcn_readlane(k, 48)));
}

// Lexicographic minimum of (d, k) over a wave's lanes, in every lane, in two
// stages: the least d, then the least k among the lanes holding it.  Equal to
// the pairwise lexicographic reduction for NaN-free d (-0 and +0 compare
// equal in both).
__device__ __forceinline__ void lap_wave_lexmin(double& d, int& k) {
  const double m = lap_wave_fmin(d);
  k = lap_wave_imin(d == m ? k : INT_MAX);
  d = m;
}

// Solves max_sigma sum_i W[i, sigma(i)] for the n x n block of W (leading
// dimension ld) with the NT threads of the calling workgroup (all must call).
// sigma: on entry the row argmax (lowest column on ties) when u_init is given,
// on exit the assignment.  u_init: -max_j W[i, j] in FP64, or null to compute
// both here.  v_part: null, or v_chunks partial column minima of c_ij - u_i
// (v_part[c * n + j]; only together with u_init).  Returns the number of rows
// unmatched after the row maxima, or -1 (sigma all -1) when W holds values
// that admit no finite path.
template <int NT>
__device__ int lap_solve(const float* __restrict__ W, int n, size_t ld, int32_t* sigma,
                         const double* u_init, const double* v_part, int v_chunks, LapArrays a,
                         LapShared<NT / 64>& sh) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const double inf = __builtin_inf();

  // ---- duals u_i = min_j c_ij = -max_j W_ij and the row argmax (lowest j)
  if (u_init != nullptr) {
    for (int i = tid; i < n; i += NT) a.u[i] = u_init[i];
  } else {
    for (int i = wave; i < n; i += NW) {
      const float* r = W + (size_t)i * ld;
      float best = -INFINITY;
      int bi = INT_MAX;
      for (int j = lane; j < n; j += 64) {
        const float x = r[j];
        if (x > best) {
          best = x;
          bi = j;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const float ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      if (lane == 0) {
        a.u[i] = -(double)best;
        sigma[i] = bi < n ? bi : -1;
      }
    }
  }
  for (int j = tid; j < n; j += NT) {
    double vj = 0.0;
    if (v_part != nullptr) {
      vj = v_part[j];
      for (int c = 1; c < v_chunks; ++c) vj = fmin(vj, v_part[(size_t)c * n + j]);
    }
    a.v[j] = vj;
    a.row_of[j] = INT_MAX;
  }
  __syncthreads();
  // ---- keep tight argmax columns; a column goes to its lowest claiming row
  for (int i = tid; i < n; i += NT) {
    const int j = sigma[i];
    if (j >= 0 && j < n && (-(double)W[(size_t)i * ld + j]) - a.u[i] - a.v[j] == 0.0)
      atomicMin(&a.row_of[j], i);
  }
  __syncthreads();
  for (int i = tid; i < n; i += NT) {
    const int j = sigma[i];
    a.col_of[i] = (j >= 0 && j < n && a.row_of[j] == i) ? j : -1;
  }
  __syncthreads();
  for (int j = tid; j < n; j += NT)
    if (a.row_of[j] == INT_MAX) a.row_of[j] = -1;

  // ---- unmatched rows in increasing order (ordered compaction)
  int nfree = 0;
  for (int base = 0; base < n; base += NT) {
    const int i = base + tid;
    const bool f = i < n && a.col_of[i] == -1;
    const unsigned long long m = __ballot(f);
    if (lane == 0) sh.cnt[wave] = __popcll(m);
    __syncthreads();
    int off = nfree;
    for (int w = 0; w < wave; ++w) off += sh.cnt[w];
    if (f) a.freel[off + __popcll(m & ((1ull << lane) - 1ull))] = i;
    for (int w = 0; w < NW; ++w) nfree += sh.cnt[w];
    __syncthreads();
  }

  const int unmatched = nfree;

  // ---- augmenting row reduction: unmatched rows bid for columns.  All
  // threads take the same decisions from the same reduced values; thread 0
  // writes the matching and the list.  A bid is a fixed amount of work, and
  // their number is bounded, so this phase always ends.
  {
    // Bids in total, over both passes: a bidding war past this is cheaper to
    // finish with shortest paths (at n = 4000 near convergence, 4 nfree + n/2
    // took 8% less time than twice as many).
    int budget = 4 * nfree + n / 2;
    for (int pass = 0; pass < 2 && nfree > 0 && budget > 0; ++pass) {
      int k = 0, nnext = 0;
      const int cnt = nfree;
      while (k < cnt) {
        if (budget <= 0) {  // carry the rows not yet seen over unchanged
          if (tid == 0)
            for (int t = k; t < cnt; ++t) a.freel[nnext + (t - k)] = a.freel[t];
          nnext += cnt - k;
          __syncthreads();
          break;
        }
        --budget;
        const int i = a.freel[k++];
        const float* ri = W + (size_t)i * ld;
        double m1 = inf, m2 = inf;
        int j1 = INT_MAX, j2 = INT_MAX;
        for (int j = tid; j < n; j += NT) {
          const double h = -(double)ri[j] - a.v[j];
          const bool b1 = lap_lex_less(h, j, m1, j1), b2 = lap_lex_less(h, j, m2, j2);
          m2 = b1 ? m1 : (b2 ? h : m2);
          j2 = b1 ? j1 : (b2 ? j : j2);
          m1 = b1 ? h : m1;
          j1 = b1 ? j : j1;
        }
        lap_wave_top2(m1, j1, m2, j2);
        if (lane == 0) {
          sh.b1[wave] = m1;
          sh.b2[wave] = m2;
          sh.c1[wave] = j1;
          sh.c2[wave] = j2;
        }
        __syncthreads();
        m1 = sh.b1[0];
        m2 = sh.b2[0];
        j1 = sh.c1[0];
        j2 = sh.c2[0];
#pragma unroll
        for (int w = 1; w < NW; ++w)
          lap_top2_merge(m1, j1, m2, j2, sh.b1[w], sh.c1[w], sh.b2[w], sh.c2[w]);
        if (j2 == INT_MAX) {  // fewer than two finite choices: left to the paths
          if (tid == 0) a.freel[nnext] = i;
          ++nnext;
          __syncthreads();
          continue;
        }
        int i0 = a.row_of[j1];
        const bool lower = m1 < m2;
        if (lower) {
          if (j1 % NT == tid) a.v[j1] -= m2 - m1;
        } else if (i0 >= 0) {
          j1 = j2;
          i0 = a.row_of[j2];
        }
        __syncthreads();  // every thread has read row_of before it changes
        if (tid == 0) {
          if (i0 >= 0) a.col_of[i0] = -1;
          a.row_of[j1] = i;
          a.col_of[i] = j1;
          a.u[i] = m2;
        }
        if (i0 >= 0) {
          if (lower) {
            --k;
            if (tid == 0) a.freel[k] = i0;
          } else {
            if (tid == 0) a.freel[nnext] = i0;
            ++nnext;
          }
        }
        __syncthreads();
      }
      nfree = nnext;
    }
  }

  // ---- one shortest augmenting path per row still unmatched
  int fail = 0;
  int par = 0;
  for (int k = 0; k < nfree; ++k) {
    const int i0 = a.freel[k];
    const double ui0 = a.u[i0];
    const float* r0 = W + (size_t)i0 * ld;
    for (int j = tid; j < n; j += NT) {
      a.dist[j] = (-(double)r0[j] - ui0) - a.v[j];
      a.pred[j] = i0;
      a.scanned[j] = 0;
    }
    int jend = -1;
    double D = 0.0;
    while (true) {
      // Closest unscanned column: each thread scans its own columns.  The
      // posted minima are double-buffered, so one barrier per step suffices.
      double bd = inf;
      int bj = INT_MAX;
      for (int j = tid; j < n; j += NT)
        if (!a.scanned[j] && a.dist[j] < bd) {
          bd = a.dist[j];
          bj = j;
        }
      lap_wave_min(bd, bj);
      if (lane == 0) {
        sh.wd[par][wave] = bd;
        sh.wj[par][wave] = bj;
      }
      __syncthreads();
      bd = sh.wd[par][0];
      bj = sh.wj[par][0];
#pragma unroll
      for (int w = 1; w < NW; ++w) lap_better(bd, bj, sh.wd[par][w], sh.wj[par][w]);
      par ^= 1;
      if (bj == INT_MAX) {  // no finite distance left
        fail = 1;
        break;
      }
      if (bj % NT == tid) a.scanned[bj] = 1;
      const int i = a.row_of[bj];
      if (i == -1) {
        jend = bj;
        D = bd;
        break;
      }
      // Relax the unscanned columns through row i (matched to column bj).
      const double ui = a.u[i];
      const float* ri = W + (size_t)i * ld;
      for (int j = tid; j < n; j += NT) {
        if (a.scanned[j]) continue;
        const double nd = ((bd + (-(double)ri[j])) - ui) - a.v[j];
        if (nd < a.dist[j]) {
          a.dist[j] = nd;
          a.pred[j] = i;
        }
      }
    }
    if (fail) break;
    // Potentials: reduced costs stay >= 0 and the path becomes tight.  Every
    // scanned column other than jend is matched to a distinct row != i0.
    for (int j = tid; j < n; j += NT) {
      if (!a.scanned[j] || j == jend) continue;
      a.v[j] += a.dist[j] - D;
      a.u[a.row_of[j]] += D - a.dist[j];
    }
    if (tid == 0) a.u[i0] += D;
    __syncthreads();
    if (tid == 0) {  // flip the path
      int j = jend;
      while (true) {
        const int i = a.pred[j];
        const int jprev = a.col_of[i];
        a.row_of[j] = i;
        a.col_of[i] = j;
        if (i == i0) break;
        j = jprev;
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += NT) sigma[i] = fail ? -1 : a.col_of[i];
  __syncthreads();
  return fail ? -1 : unmatched;
}

// ---------------------------------------------------------------------------
// Parallel bidding: a Jacobi form of the augmenting row reduction above.  In
// one round every unmatched row bids at once against the same column prices:
// it finds its best and second-best reduced costs m1 <= m2 (columns j1, j2)
// and asks for j1 with the price drop m2 - m1, or, when m1 == m2 and j1 is
// taken, for j2 without a drop -- the choice a sequential bid makes.  Each
// column goes to its largest bid (ties: the lowest row); the winner takes it
// with u_i = m2, the column's price falls by the winner's drop, and the
// displaced owner becomes unmatched.  Prices only fall and every winner's
// column falls by its own drop alone, so the invariants of the sequential
// version hold (every reduced cost >= 0, matched pairs tight); the rows left
// unmatched when the rounds stop (none left, or no progress for a few rounds)
// go to the shortest augmenting paths, which make the result exact.  Which
// rows bid in a round is a set, and a column's winner depends only on the
// bids, so the outcome does not depend on the order of the lists.
struct LapBidState {
  double* u;
  double* v;
  int* row_of;
  int* col_of;
  int* list[2];             // unmatched rows of the current / next round
  unsigned long long* key;  // per column: the round's best bid (0: none)
  int* tgt;                 // per row: the column it bid for (-1: no bid)
  double* newu;             // per row: its u if it wins (m2)
  double* drop;             // per row: its column's price drop if it wins
  int* ctl;                 // [0..1] list counts, [2] stop, [3] best count, [4] stalled
                            // rounds, [6] rows the row maxima left free, [7] workgroups
                            // done with the current round
};

// Rounds without a smaller unmatched count after which bidding stops.
constexpr int kBidStall = 8;


__device__ __forceinline__ unsigned long long lap_bid_key(double d, int i) {
  // Larger drops first, then lower rows; d >= 0 (or +inf), so the FP32 bit
  // pattern orders like the value.
  const float f = (float)d;
  return ((unsigned long long)__float_as_uint(f) << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned)i);
}

// One wave per unmatched row of list `p`: the row's bid.
__device__ inline void lap_bid_row(const float* __restrict__ W, int n, size_t ld,
                                   const LapBidState& s, int i) {
  const int lane = threadIdx.x & 63;
  const double inf = __builtin_inf();
  const float* ri = W + (size_t)i * ld;
  // Best two (value, column) pairs of this lane's columns: four independent
  // chains (columns j, j + 64, j + 128, j + 192 of each 256-column block) so
  // that four reads and comparisons are in flight, merged at the end (the
  // columns are distinct, so the best two do not depend on the order).
  double m1[4], m2[4];
  int j1[4], j2[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    m1[t] = m2[t] = inf;
    j1[t] = j2[t] = INT_MAX;
  }
  auto take = [&](int t, int j) {
    const double h = -(double)ri[j] - s.v[j];
    const bool b1 = lap_lex_less(h, j, m1[t], j1[t]), b2 = lap_lex_less(h, j, m2[t], j2[t]);
    m2[t] = b1 ? m1[t] : (b2 ? h : m2[t]);
    j2[t] = b1 ? j1[t] : (b2 ? j : j2[t]);
    m1[t] = b1 ? h : m1[t];
    j1[t] = b1 ? j : j1[t];
  };
  int j = lane;
  for (; j + 192 < n; j += 256) {
#pragma unroll
    for (int t = 0; t < 4; ++t) take(t, j + 64 * t);
  }
  for (; j < n; j += 64) take(0, j);
#pragma unroll
  for (int t = 1; t < 4; ++t) lap_top2_merge(m1[0], j1[0], m2[0], j2[0], m1[t], j1[t], m2[t], j2[t]);
  double b1 = m1[0], b2 = m2[0];
  int c1 = j1[0], c2 = j2[0];
  lap_wave_top2(b1, c1, b2, c2);
  if (lane == 0) {
    if (c2 == INT_MAX) {  // fewer than two finite choices: left to the paths
      __hip_atomic_store(&s.tgt[i], -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    const bool lower = b1 < b2;
    int target = c1;
    if (!lower && s.row_of[c1] >= 0) target = c2;
    const double d = lower ? b2 - b1 : 0.0;
    // Read back by the workgroup that resolves the round: written through
    // to the device-coherent level (agent scope), as is the key.
    __hip_atomic_store(&s.tgt[i], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&s.newu[i], b2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&s.drop[i], d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    atomicMax(&s.key[target], lap_bid_key(d, i));
  }
}

// After the bids of a round: row i of list p takes its column if its bid won
// (and resets the column's key for the next round), else stays unmatched.
// The bids of the round were made by other workgroups: read at the
// device-coherent level (agent scope).
__device__ inline void lap_resolve_row(const LapBidState& s, int i, int q) {
  const int j = __hip_atomic_load(&s.tgt[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int again = i;
  const double di = __hip_atomic_load(&s.drop[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (j >= 0 && __hip_atomic_load(&s.key[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                    lap_bid_key(di, i)) {
    const int i0 = s.row_of[j];
    s.v[j] -= di;
    s.row_of[j] = i;
    s.col_of[i] = j;
    s.u[i] = __hip_atomic_load(&s.newu[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s.key[j] = 0;
    again = i0;
    if (i0 >= 0) s.col_of[i0] = -1;
  }
  if (again >= 0) s.list[q][atomicAdd(&s.ctl[q], 1)] = again;
}

// ---------------------------------------------------------------------------
// The same solver with the column state in registers, for n <= NT * C and a
// given row reduction (u_init, v_part).  Thread t owns the C consecutive
// columns t*C ... t*C + C - 1 and keeps their prices v, tentative distances
// and scanned flags in registers; the row duals u, the matching, the
// predecessors and the unmatched-row list stay in LDS.  lap_solve spends most
// of a Dijkstra step or bid on work that every one of its 16 waves repeats
// (the wave reductions, the merge of the posted minima, LDS reads of the
// column arrays); with one wave per SIMD and the columns in registers that
// work is done once per SIMD.  The rules, the FP64 arithmetic of every
// distance and potential, and the tie order (lowest column) are those of
// lap_solve: the minimum and best-two of a row do not depend on how its
// columns are split over threads, so both give the same assignment.
struct LapRegArrays {
  double* u;      // row duals
  double* vinit;  // column prices at the start (read across threads once)
  int* row_of;
  int* col_of;
  int* pred;
  int* freel;
};

__host__ __device__ inline size_t lap_reg_lds_bytes(int n) {
  return ((size_t)n * (2 * 8 + 4 * 4) + 15) / 16 * 16;
}

__device__ inline LapRegArrays lap_reg_carve(char* base, int n) {
  LapRegArrays a;
  a.u = reinterpret_cast<double*>(base);
  a.vinit = a.u + n;
  a.row_of = reinterpret_cast<int*>(a.vinit + n);
  a.col_of = a.row_of + n;
  a.pred = a.col_of + n;
  a.freel = a.pred + n;
  return a;
}

// Row i's entries in this thread's columns (0 past n); float4 loads where the
// row is 16-byte aligned and the thread's columns all lie inside it.
template <int C>
__device__ __forceinline__ void lap_row_cols(const float* __restrict__ row, int j0, int n, bool vec,
                                             float (&x)[C]) {
  if (vec && j0 + C <= n) {
#pragma unroll
    for (int q = 0; q < C / 4; ++q) {
      const float4 t = *reinterpret_cast<const float4*>(row + j0 + 4 * q);
      x[4 * q] = t.x;
      x[4 * q + 1] = t.y;
      x[4 * q + 2] = t.z;
      x[4 * q + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = (j0 + c < n) ? row[j0 + c] : 0.0f;
  }
}

// Row i's entries in this thread's columns, the same for every thread: C / 4
// float4 reads, those of column groups past n clamped to the row's last four
// columns (their values are never used: such columns enter every search as
// scanned, at distance inf).  Needs n % 4 == 0, n >= 4 and 16-byte aligned
// rows.  With no per-thread branch, a read issued ahead stays in flight until
// its registers are used.
template <int C>
__device__ __forceinline__ void lap_row_cols4(const float* __restrict__ row, int j0, int n,
                                              float (&x)[C]) {
#pragma unroll
  for (int q = 0; q < C / 4; ++q) {
    const int jj = (j0 + 4 * q < n) ? j0 + 4 * q : n - 4;
    const float4 t = *reinterpret_cast<const float4*>(row + jj);
    x[4 * q] = t.x;
    x[4 * q + 1] = t.y;
    x[4 * q + 2] = t.z;
    x[4 * q + 3] = t.w;
  }
}

// V4: rows read by lap_row_cols4 (the caller checks its conditions).
template <int NT, int C, bool V4>
__device__ int lap_solve_reg(const float* __restrict__ W, int n, size_t ld, int32_t* sigma,
                             const double* __restrict__ u_init, const double* v_part,
                             int v_chunks, LapRegArrays a, LapShared<NT / 64>& sh,
                             const LapBidState* given = nullptr) {
  static_assert(C % 4 == 0 && C <= 32, "columns per thread");
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const double inf = __builtin_inf();
  const int j0 = tid * C;
  const bool vec = (ld % 4 == 0) && ((reinterpret_cast<uintptr_t>(W) & 15) == 0);
  auto load_row = [&](int r, float(&dst)[C]) {
    if constexpr (V4)
      lap_row_cols4<C>(W + (size_t)r * ld, j0, n, dst);
    else
      lap_row_cols<C>(W + (size_t)r * ld, j0, n, vec, dst);
  };

  double v[C];
  if (given != nullptr) {
    // The state left by the parallel bidding rounds: duals and matching.
    for (int i = tid; i < n; i += NT) {
      a.u[i] = given->u[i];
      a.row_of[i] = given->row_of[i];
      a.col_of[i] = given->col_of[i];
    }
#pragma unroll
    for (int c = 0; c < C; ++c) v[c] = (j0 + c < n) ? given->v[j0 + c] : 0.0;
    __syncthreads();
  } else {
  // ---- duals: u_i = -max_j W_ij (given), v_j = min of the partial column
  // minima (or 0)
  for (int i = tid; i < n; i += NT) a.u[i] = u_init[i];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int j = j0 + c;
    double vj = 0.0;
    if (j < n) {
      if (v_part != nullptr) {
        vj = v_part[j];
        for (int k = 1; k < v_chunks; ++k) vj = fmin(vj, v_part[(size_t)k * n + j]);
      }
      a.vinit[j] = vj;
      a.row_of[j] = INT_MAX;
    }
    v[c] = vj;
  }
  __syncthreads();
  // ---- keep tight argmax columns; a column goes to its lowest claiming row
  for (int i = tid; i < n; i += NT) {
    const int j = sigma[i];
    if (j >= 0 && j < n && (-(double)W[(size_t)i * ld + j]) - a.u[i] - a.vinit[j] == 0.0)
      atomicMin(&a.row_of[j], i);
  }
  __syncthreads();
  for (int i = tid; i < n; i += NT) {
    const int j = sigma[i];
    a.col_of[i] = (j >= 0 && j < n && a.row_of[j] == i) ? j : -1;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < C; ++c)
    if (j0 + c < n && a.row_of[j0 + c] == INT_MAX) a.row_of[j0 + c] = -1;
  }

  // Columns of this thread still unmatched (bit c: column j0 + c).  Among
  // columns at the same tentative distance the path search takes an
  // unmatched one first: any column of least distance may end a shortest
  // path, and on tie-heavy matrices (a constant N, as after one outer
  // iteration) this ends each search at once instead of after scanning every
  // matched column of that distance.
  unsigned freecols = 0;
#pragma unroll
  for (int c = 0; c < C; ++c)
    if (j0 + c < n && a.row_of[j0 + c] == -1) freecols |= 1u << c;

  // ---- unmatched rows in increasing order (ordered compaction)
  int nfree = 0;
  for (int base = 0; base < n; base += NT) {
    const int i = base + tid;
    const bool f = i < n && a.col_of[i] == -1;
    const unsigned long long m = __ballot(f);
    if (lane == 0) sh.cnt[wave] = __popcll(m);
    __syncthreads();
    int off = nfree;
    for (int w = 0; w < wave; ++w) off += sh.cnt[w];
    if (f) a.freel[off + __popcll(m & ((1ull << lane) - 1ull))] = i;
    for (int w = 0; w < NW; ++w) nfree += sh.cnt[w];
    __syncthreads();
  }
  const int unmatched = given != nullptr ? given->ctl[6] : nfree;

  // ---- augmenting row reduction (bids), as in lap_solve; none after the
  // parallel rounds
  float x[C];
  {
    int budget = given != nullptr ? 0 : 4 * nfree + n / 2;
    for (int pass = 0; pass < 2 && nfree > 0 && budget > 0; ++pass) {
      int k = 0, nnext = 0;
      const int cnt = nfree;
      while (k < cnt) {
        if (budget <= 0) {
          if (tid == 0)
            for (int t = k; t < cnt; ++t) a.freel[nnext + (t - k)] = a.freel[t];
          nnext += cnt - k;
          __syncthreads();
          break;
        }
        --budget;
        const int i = a.freel[k++];
        load_row(i, x);
        double m1 = inf, m2 = inf;
        int j1 = INT_MAX, j2 = INT_MAX;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          // Columns past n take part as (inf, INT_MAX), which never ranks
          // above "no choice", so they can never be bid for.
          const int j = (j0 + c < n) ? j0 + c : INT_MAX;
          const double h = (j != INT_MAX) ? -(double)x[c] - v[c] : inf;
          const bool b1 = lap_lex_less(h, j, m1, j1), b2 = lap_lex_less(h, j, m2, j2);
          m2 = b1 ? m1 : (b2 ? h : m2);
          j2 = b1 ? j1 : (b2 ? j : j2);
          m1 = b1 ? h : m1;
          j1 = b1 ? j : j1;
        }
        lap_wave_top2(m1, j1, m2, j2);
        if (lane == 0) {
          sh.b1[wave] = m1;
          sh.b2[wave] = m2;
          sh.c1[wave] = j1;
          sh.c2[wave] = j2;
        }
        __syncthreads();
        m1 = sh.b1[0];
        m2 = sh.b2[0];
        j1 = sh.c1[0];
        j2 = sh.c2[0];
#pragma unroll
        for (int w = 1; w < NW; ++w)
          lap_top2_merge(m1, j1, m2, j2, sh.b1[w], sh.c1[w], sh.b2[w], sh.c2[w]);
        if (j2 == INT_MAX) {  // fewer than two finite choices: left to the paths
          if (tid == 0) a.freel[nnext] = i;
          ++nnext;
          __syncthreads();
          continue;
        }
        int i0 = a.row_of[j1];
        const bool lower = m1 < m2;
        if (lower) {
#pragma unroll
          for (int c = 0; c < C; ++c)
            if (j0 + c == j1) v[c] -= m2 - m1;
        } else if (i0 >= 0) {
          j1 = j2;
          i0 = a.row_of[j2];
        }
        __syncthreads();  // every thread has read row_of before it changes
        if (tid == 0) {
          if (i0 >= 0) a.col_of[i0] = -1;
          a.row_of[j1] = i;
          a.col_of[i] = j1;
          a.u[i] = m2;
        }
        if (j1 >= j0 && j1 < j0 + C) freecols &= ~(1u << (j1 - j0));
        if (i0 >= 0) {
          if (lower) {
            --k;
            if (tid == 0) a.freel[k] = i0;
          } else {
            if (tid == 0) a.freel[nnext] = i0;
            ++nnext;
          }
        }
        __syncthreads();
      }
      nfree = nnext;
    }
  }

  // ---- one shortest augmenting path per row still unmatched
  //
  // Each step scans the column of least tentative distance and relaxes the
  // unscanned columns through the row matched to it, whose entries are a
  // dependent read of W.  Most often (three steps in four on the n = 4000
  // workloads) the next step's column is the best one outside the thread that
  // holds this step's column, so that column's row is read ahead, during the
  // relaxation and the next step's search, and used when the guess was right.
  // The guess only decides what is read early: the path is the same.
  int fail = 0;
  int par = 0;
  float xs[C];  // the second row buffer of the path search
  for (int k = 0; k < nfree; ++k) {
    const int i0 = a.freel[k];
    const double ui0 = a.u[i0];
    load_row(i0, x);
    double dist[C];
    int pr[C];  // predecessor rows, kept here until the path is complete
    unsigned scanned = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = j0 + c;
      pr[c] = i0;
      if (j < n) {
        dist[c] = (-(double)x[c] - ui0) - v[c];
      } else {
        dist[c] = inf;
        scanned |= 1u << c;
      }
    }
    int ipre = -1;
    int jend = -1;
    double D = 0.0;
    // One step of the search.  cur holds row ipre's entries, read ahead by
    // the previous step; nxt receives the read ahead for the next one.  The
    // steps alternate the two buffers, so a read ahead lands in the registers
    // it is used from (no copy that would wait for it).  Returns 0 to go on,
    // 1 when the path ends at an unmatched column, 2 when no finite distance
    // is left.
    auto step = [&](float(&cur)[C], float(&nxt)[C]) -> int {
      // This thread's least unscanned column.  Order: distance, then
      // unmatched before matched, then column (key j for an unmatched column,
      // n + j for a matched one).  Scanned columns and NaN distances enter as
      // (inf, INT_MAX), as in a scan that takes a column only when it is
      // lexicographically below the best so far, starting from (inf,
      // INT_MAX).  The minimum in two stages: the least distance (a tree),
      // then the least key among the columns at that distance.
      double td[C];
      int tk[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const bool open = !((scanned >> c) & 1u) && !__builtin_isnan(dist[c]);
        td[c] = open ? dist[c] : inf;
        tk[c] = open ? (((freecols >> c) & 1u) ? j0 + c : n + j0 + c) : INT_MAX;
      }
      double dm[C];
#pragma unroll
      for (int c = 0; c < C; ++c) dm[c] = td[c];
#pragma unroll
      for (int h = 1; h < C; h *= 2)
#pragma unroll
        for (int c = 0; c + h < C; c += 2 * h) dm[c] = fmin(dm[c], dm[c + h]);
      const double tmin = dm[0];
      int km[C];
#pragma unroll
      for (int c = 0; c < C; ++c) km[c] = td[c] == tmin ? tk[c] : INT_MAX;
#pragma unroll
      for (int h = 1; h < C; h *= 2)
#pragma unroll
        for (int c = 0; c + h < C; c += 2 * h) km[c] = min(km[c], km[c + h]);
      const int kmin = km[0];
      // The wave's least column, then its least outside the thread holding
      // that one (the read-ahead guess).
      double bd = tmin;
      int bj = kmin;
      lap_wave_lexmin(bd, bj);
      const bool mine = kmin == bj;
      double gd = mine ? inf : tmin;
      int gj = mine ? INT_MAX : kmin;
      lap_wave_lexmin(gd, gj);
      if (lane == 0) {
        sh.wd[par][wave] = bd;
        sh.wj[par][wave] = bj;
        sh.w2d[par][wave] = gd;
        sh.w2j[par][wave] = gj;
      }
      __syncthreads();
      bd = sh.wd[par][0];
      bj = sh.wj[par][0];
      gd = sh.w2d[par][0];
      gj = sh.w2j[par][0];
#pragma unroll
      for (int w = 1; w < NW; ++w)
        lap_top2_merge(bd, bj, gd, gj, sh.wd[par][w], sh.wj[par][w], sh.w2d[par][w],
                       sh.w2j[par][w]);
      par ^= 1;
      if (bj == INT_MAX) return 2;
      if (bj >= n) bj -= n;
      if (bj >= j0 && bj < j0 + C) scanned |= 1u << (bj - j0);
      const int i = a.row_of[bj];
      if (i == -1) {
        jend = bj;
        D = bd;
        return 1;
      }
      // Row i (matched to column bj): already in cur when the last guess
      // named it, else read now; then read ahead the guess for the next
      // step, the row matched to column gj (row i again when there is none:
      // a read that is never used, but every path then issues the same
      // reads, so waiting for cur never waits for the read ahead).
      int inext = -1;
      if (gj != INT_MAX) {
        const int g = gj >= n ? gj - n : gj;
        if (g >= 0 && g < n) inext = a.row_of[g];
      }
      const double ui = a.u[i];
      if (i != ipre) load_row(i, cur);
      ipre = (inext >= 0 && inext < n) ? inext : i;
      load_row(ipre, nxt);
      // Relax the unscanned columns through row i.
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const double nd = ((bd + (-(double)cur[c])) - ui) - v[c];
        const bool upd = !((scanned >> c) & 1u) && nd < dist[c];
        dist[c] = upd ? nd : dist[c];
        pr[c] = upd ? i : pr[c];
      }
      return 0;
    };
    int r;
    while (true) {
      if ((r = step(x, xs)) != 0) break;
      if ((r = step(xs, x)) != 0) break;
    }
    if (r == 2) fail = 1;
    if (fail) break;
    // Predecessors to LDS for the flip, and the potentials, as in lap_solve.
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int j = j0 + c;
      if (j < n) a.pred[j] = pr[c];
      if (!((scanned >> c) & 1u) || j >= n || j == jend) continue;
      v[c] += dist[c] - D;
      a.u[a.row_of[j]] += D - dist[c];
    }
    if (tid == 0) a.u[i0] += D;
    if (jend >= j0 && jend < j0 + C) freecols &= ~(1u << (jend - j0));
    __syncthreads();
    if (tid == 0) {  // flip the path
      int j = jend;
      while (true) {
        const int i = a.pred[j];
        const int jprev = a.col_of[i];
        a.row_of[j] = i;
        a.col_of[i] = j;
        if (i == i0) break;
        j = jprev;
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += NT) sigma[i] = fail ? -1 : a.col_of[i];
  __syncthreads();
  return fail ? -1 : unmatched;
}

}  // namespace fram
