// Internal declarations shared by the HIP translation units of libfram.
// Nothing here is part of the public ABI (see include/fram.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace fram {

// ----------------------------------------------------------------------------
// Device-visible scalar state of one solve.  Lives in device memory; the host
// reads it back with one async copy per outer iteration.
struct DevState {
  int done;          // SDSN converged (or capped) for the current projection
  int passes;        // SDSN passes made by the current projection
  int invalid;       // flags: 1 non-finite, 2 negative, 4 asymmetric input; 8 barrier
                     // timeout, 16 on-chip roll call failed (on-chip SDSN)
  int total_passes;  // passes summed over projections (on-chip SDSN path)
  int max_passes;    // largest pass count of one projection (on-chip SDSN path)
  int capped;        // some projection hit the pass cap (on-chip SDSN path)
  int lap_paths;     // augmenting paths of the final assignment (-1: failed)
  double gamma;      // gamma of the last SDSN output
  double delta;      // delta of the last outer update
  double dnum;       // ||N_new - N_old||_F^2 of the last update
  double dden;       // ||N_new||_F^2 of the last update
  double maxA;       // max entry of A (unscaled)
  double maxB;       // max entry of B (unscaled)
  double maxK;       // max |entry| of the node similarities K (unscaled)
  double objective;  // sum_{k,l} A_kl B_{s(k)s(l)}
  double nmax;       // max of N after the last update (DSPFP criterion)
  double nmax_prev;  // ... and before it
};

// One set of tile partials over an np x np matrix cut into nb x nb tiles of
// edge BM (np = nb * BM), all sums in FP64.  rowp[bn * np + i] = sum over the
// columns of tile column bn of row i; colp[bm * np + j] = sum over the rows of
// tile row bm of column j; tot[bm * nb + bn] = total of tile (bm, bn);
// tmax = FP32 tile max.
struct Partials {
  double* rowp;
  double* colp;
  double* tot;
  float* tmax;
};

enum class Elem : int { F32 = 0, BF16 = 1, F16 = 2 };

inline size_t elem_size(Elem e) { return e == Elem::F32 ? 4 : 2; }

// ------------------------------------------------------------------ launches
// All launches are asynchronous on `s`; they return hipSuccess or the launch
// error.  Matrices are row-major with leading dimension ld (elements).

// C (np x np) = P (np x np) * Q^T over K = n (rounded up to the K step),
// inputs of type e, FP32 accumulation.
// C is written as type e when c_f32 == false, as float otherwise; with
// c_f32, an optional FP32 matrix `bias` (same layout as C) is added to every
// output.  np must be a multiple of bm (64, 128 or 256); all padding
// rows/columns of P and Q must be zero up to np.
hipError_t launch_gemm_nt(Elem e, int bm, const void* P, const void* Q, void* C, bool c_f32,
                          int n, int np, int ld, hipStream_t s, const float* bias = nullptr);

// ---------------------------------------------------------- group launches
// The per-iteration kernels of many small pairs in one launch each, one job
// per pair (device arrays of jobs).  Every pair's matrix is a single tile
// (np == bm), and each job is computed exactly as the corresponding
// single-pair launch would compute it.

struct GemmJob {  // C = P * Q^T over K = n
  const void* P;
  const void* Q;
  void* C;
  int ld;      // leading dimension (np)
  int ktiles;  // gemm_ktiles(e, n)
};
int gemm_ktiles(Elem e, int n);
// All jobs have np == bm.  Output as launch_gemm_nt with the same c_f32.
hipError_t launch_gemm_group(Elem e, int bm, bool c_f32, const GemmJob* jobs, int count,
                             hipStream_t s);

struct SdsnJob {  // one projection: statistics of X, then every pass, in place
  float* X;
  int n, np;
  Partials p0, p1;
  DevState* st;
};
// Jobs with np == bm; same iterates as launch_tile_stats + launch_sdsn_chunk.
hipError_t launch_sdsn_group(int bm, const SdsnJob* jobs, int count, int max_passes,
                             double theta, double gamma_tol, hipStream_t s);

struct UpdateJob {  // N <- (1-alpha) N + alpha D, the GEMM-type copy, delta
  const float* D;
  float* N;
  void* Nlp;
  int n, np, nblocks;  // nblocks = update_blocks(n), as the single-pair launch
  double* part;
  DevState* st;
};
hipError_t launch_update_group(Elem e, const UpdateJob* jobs, int count, int max_blocks,
                               double alpha, hipStream_t s);

// Tile statistics of an n x n matrix: reads src (ld_src), writes it padded to
// dst (np x np, ld np, zero padding) unless dst == nullptr or dst == src, and
// fills `out` (row/col partials, FP64 tile totals, tile maxima).  Also resets
// the SDSN fields of *st.
hipError_t launch_tile_stats(int bm, const float* src, int ld_src, float* dst, int n, int np,
                             Partials out, DevState* st, hipStream_t s);

// Passes k_first .. k_last of a projection whose padded matrix is one tile
// (np == bm), in a single workgroup launch; p0 / p1 are the partial buffers of
// even / odd pass parity (pass k reads parity k - 1, writes parity k).
hipError_t launch_sdsn_chunk(int bm, float* X, int n, int np, Partials p0, Partials p1,
                             DevState* st, int k_first, int k_last, int max_passes, double theta,
                             double gamma_tol, hipStream_t s, double fixed_scale = 0.0);
// One SDSN pass (Algorithm 2 body) over X in place, pass index k >= 1.  Reads
// the partials of its input from `in`, writes those of its output to `out`.
hipError_t launch_sdsn_pass(int bm, float* X, int n, int np, Partials in, Partials out,
                            DevState* st, int k, int max_passes, double theta,
                            double gamma_tol, hipStream_t s, double fixed_scale = 0.0);

// Bits of DevState::invalid set by the on-chip SDSN.
constexpr int kInvalidBarrier = 8;    // a grid barrier timed out (launch aborted)
constexpr int kInvalidRollCall = 16;  // not all workgroups became resident: nothing done
// Largest on-chip grid (workgroups) the synchronisation counters allow.
constexpr long kOnchipMaxGrid = 4096;
// Bytes of the synchronisation block of one on-chip launch (zeroed before it).
constexpr size_t kOnchipSyncBytes = 2048;

// Arguments of the on-chip SDSN projection (sdsn_onchip.hip).
struct OnchipArgs {
  const float* src;  // input matrix, leading dimension ld_src
  int ld_src;
  int src_vec;       // 1: rows of src are 16-byte aligned (float4 loads)
  float* dst;        // optional: final D, np x np (ld np); nullptr to skip
  int n, np;
  Partials p[2];     // ping-pong partial sets (set 0 also gets tile maxima)
  DevState* st;
  unsigned* sync;    // kOnchipSyncBytes, zero at launch: barrier counters, abort flag
  long long roll_ticks;  // bound (wall-clock ticks) on the roll call
  long long wait_ticks;  // bound on every later barrier wait
  int max_passes;
  double theta, gamma_tol;
  float* N;          // optional fused update: N <- (1-alpha) N + alpha D
  void* Nlp;         // GEMM-type copy of N (nlp_kind 1 = bf16, 2 = f16, 0 = none)
  int nlp_kind;
  float alpha;
  double* dpart;     // FP64 delta partials, 2 per workgroup (tile order)
};

// Workgroups of the BM variant that fit on one compute unit (0 on error).
int sdsn_onchip_per_cu(int bm);

// True if the nb*nb workgroups of the BM variant can all be resident on
// `device` at once (an idle device; the roll call covers the rest).
bool sdsn_onchip_fits(int device, int bm, int np);

// Every SDSN pass of one projection in one launch (grid nb*nb).  The caller
// zeroes a.sync on the same stream first and orders these launches across
// streams (see runtime.hip).
hipError_t launch_sdsn_onchip(int bm, const OnchipArgs& a, hipStream_t s);

// st->delta from `nblocks` pairs of FP64 partial sums (num, den).
hipError_t launch_delta_final(const double* part, int nblocks, DevState* st, hipStream_t s);

// N <- (1-alpha) N + alpha D with FP64 partial sums for delta; writes the
// GEMM-operand copy Nlp in type e (skipped when e == F32 and Nlp == N).
hipError_t launch_update(Elem e, const float* D, float* N, void* Nlp, int n, int np,
                         double alpha, double* part, int nblocks, DevState* st,
                         hipStream_t s);
int update_blocks(int n);

// Max of A and B (n x n FP64, ld n) into st->maxA / st->maxB, via partials.
hipError_t launch_maxes(const double* A, const double* B, int n, double* part, int nblocks,
                        DevState* st, hipStream_t s);
int max_blocks(int n);

// dst (np x np, type e) = src (n x n FP64) / max, zero padding.  which = 0
// uses st->maxA, 1 uses st->maxB.
hipError_t launch_cast_scaled(Elem e, const double* src, int n, void* dst, int np,
                              const DevState* st, int which, hipStream_t s);

// Node term of the gradient: dst (np x np FP32) = w K / (maxA maxB), the
// node similarities on the same scale as the scaled edge term (falls back to
// w K / max|K| when a graph has no edges), zero padding.  Computes st->maxK.
hipError_t launch_node_term(const double* K, int n, double w, float* dst, int np, double* part,
                            int nblocks, DevState* st, hipStream_t s);
// st->objective += 2 w sum_k K[k, sigma(k)] (FP64), after launch_objective.
hipError_t launch_node_objective(const double* K, const int32_t* sigma, int n, double w,
                                 DevState* st, hipStream_t s);

// dst (np x np, type e) = src (n x n float, ld n), no scaling, zero padding.
hipError_t launch_cast_f32(Elem e, const float* src, int n, void* dst, int np, hipStream_t s);

// Zero `bytes` bytes of device memory with a fill kernel.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// Validation of device inputs: sets bits of st->invalid.
hipError_t launch_validate(const double* A, int n, DevState* st, hipStream_t s);

// sigma[i] = argmax_j N[i, j] (lowest j on ties), i < n; if u is not null,
// also u[i] = -max_j N[i, j] in FP64 (the assignment's starting duals).
hipError_t launch_row_argmax(const float* N, int n, int np, int32_t* sigma, hipStream_t s,
                             double* u = nullptr);

// st->objective = sum_{k,l} A_kl B_{sigma(k) sigma(l)} in FP64.
hipError_t launch_objective(const double* A, const double* B, const int32_t* sigma, int n,
                            double* part, int nblocks, DevState* st, hipStream_t s);
int objective_blocks(int n);

// DSPFP's outer criterion (App. B.2): st->delta =
// max_ij |N_ij / max N - P_ij / max P| over the n x n block (ld np), N the
// iterate after the update and P the one before it; st->nmax_prev takes the
// previous st->nmax and st->nmax the max of N.  +inf while a maximum is not
// positive.
hipError_t launch_dspfp_criterion(const float* N, const float* P, int n, int np, double* part,
                                  int nblocks, DevState* st, hipStream_t s);

// Copy an n x n float block between leading dimensions.
hipError_t launch_copy_f32(const float* src, int ld_src, float* dst, int ld_dst, int n,
                           hipStream_t s);

// ------------------------------------------------------- device assignment
// One exact linear assignment problem: maximise sum_i w[i, sigma(i)] over
// permutations, w n x n row-major FP32 (leading dimension ld).  sigma
// receives the optimal assignment (all -1 if w admits no finite one); on
// entry it must hold the row argmax of w (lowest column on ties) when
// u_ready is set, and u_init[i] = -max_j w[i, j] in FP64 (may point into ws);
// otherwise the kernel computes both (and skips the column reduction, which
// needs u).  ws: lap_workspace_bytes(n) bytes of device memory.  paths_out
// (may be null) receives the number of rows left unmatched by the row argmax
// (0 when it is a permutation), or -1.
struct LapProblem {
  const float* w;
  int n, ld;
  int32_t* sigma;
  char* ws;
  const double* u_init;
  int u_ready;
  int* paths_out;
};
size_t lap_workspace_bytes(int n);
// Solves `count` problems, one workgroup each: either the single problem
// *one (count == 1) or the device array probs.  max_n bounds every n.
hipError_t launch_lap(const LapProblem* one, const LapProblem* probs, int count, int max_n,
                      hipStream_t s);

}  // namespace fram
