/*
 * fram.h -- C ABI of the MI355X (gfx950) FRAM library, libfram.so.
 *
 * FRAM (Frobenius-Regularized Assignment Matching) matches two graphs with
 * nonnegative symmetric edge matrices A and B (Sec. 3, "Graph") by the
 * projected fixed-point iteration of eq. (3):
 *
 *     X = A N B                      (gradient of eq. (1) without node term)
 *     D = SDSN(X, theta)             (Algorithm 2: scaled doubly stochastic
 *                                     normalisation, solves the FRA problem
 *                                     of Theorem 1)
 *     N = (1 - alpha) N + alpha D    (Algorithm 1, step 7)
 *     delta = ||N_new - N_old||_F / ||N_new||_F   (App. B.2)
 *
 * and then discretises N to a permutation by the linear assignment of eq. (2)
 * (Algorithm 1, step 10).  The GEMMs run on MFMA in FP32, BF16 or FP16 with
 * FP32 accumulation; SDSN runs in FP32 with FP64 totals for gamma; delta and
 * the final objective are accumulated in FP64.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are dense, row-major, n x n, leading dimension n unless an
 *   explicit ld argument is given.
 * - "theta" is the FRA strength of Theorem 1 (regulariser 1/theta); the
 *   argument is named lambda where it plays that role at the boundary.  The
 *   paper's node-term weight multiplies F F~^T, which this library does not
 *   take (graphs without node attributes).
 * - perm_out[i] = node of B matched to node i of A (M[i, perm_out[i]] = 1).
 * - objective_out = sum_{k,l} A[k,l] * B[perm[k], perm[l]] = tr(A M B M^T),
 *   i.e. 2 * Phi(M) of eq. (1) without node term, on the unscaled inputs,
 *   accumulated in FP64.
 * - Ownership: the caller owns every buffer it passes, host or device; the
 *   library copies inputs in and writes outputs into caller storage and never
 *   frees caller memory.  The library owns its device workspace, which lives
 *   in the context and is released by fram_destroy.
 * - Errors: return codes only.  Argument validation (NULL pointers, sizes,
 *   non-finite/negative/asymmetric host inputs, theta <= 0, iters < 1,
 *   tol < 0, HBM budget) happens before any device call.  Reaching an
 *   iteration cap is not an error: the result is returned and the stats say
 *   converged = 0 / sdsn_capped = 1.  A NaN/Inf in gamma or delta returns
 *   FRAM_ENUMERIC; a HIP runtime failure returns FRAM_EDEVICE with the text in
 *   fram_last_error().
 * - Threading: one context per host thread.  A context is not re-entrant.
 */
#ifndef FRAM_H
#define FRAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FRAM_OK = 0,
  FRAM_EINVAL = 1,    /* invalid argument (checked before any device call)   */
  FRAM_ENOMEM = 2,    /* problem exceeds the context's HBM budget            */
  FRAM_EDEVICE = 3,   /* HIP runtime error; see fram_last_error()            */
  FRAM_ENUMERIC = 4,  /* NaN/Inf met in gamma, delta or the objective        */
  FRAM_EBUSY = 5      /* server queue full / slot unavailable                */
} fram_status;

/* Input type of the two GEMMs of Algorithm 1 step 5.  SDSN always runs in FP32
 * and delta / objective in FP64 (the precision map of Algorithm 1, App. E,
 * with TF32 replaced by FP16 or BF16, which gfx950 MFMA provides). */
typedef enum { FRAM_FP32 = 0, FRAM_BF16 = 1, FRAM_FP16 = 2 } fram_precision;

/* Largest n any entry point takes (FRAM_EINVAL above it): the padded n x n
 * FP32 iterate must stay below 4 GiB, the range of the kernels' 32-bit
 * element offsets.  The workspace at this size is about 40 GB. */
#define FRAM_MAX_N 32768

typedef struct {
  int outer_iters;       /* outer iterations run (Algorithm 1 loop)                    */
  int sdsn_passes;       /* SDSN passes summed over all outer iterations               */
  int sdsn_passes_last;  /* passes of the last outer iteration                         */
  int sdsn_passes_max;   /* largest pass count of any outer iteration                  */
  int converged;         /* 1 if delta <= tol stopped the loop                         */
  int sdsn_capped;       /* 1 if some SDSN call hit sdsn_max with gamma > gamma_tol    */
  int lap_paths;         /* augmenting paths the final assignment needed: 0 when the row
                            argmax of N was already a permutation (see fram_assign)   */
  int gemm_tile;         /* GEMM / SDSN tile edge used (64, 128 or 256)                 */
  double delta;          /* last delta (App. B.2)                                      */
  double gamma;          /* gamma of the last SDSN output (Sec. 5.2)                   */
  double ms_total;       /* wall time of the call on the host, milliseconds            */
  /* Filled only when fram_options.profile is 1 or 2 (HIP events around each
   * launch on the solve's stream): summed device milliseconds and launch counts.
   * profile = 1 waits for every launch (each time is that launch alone);
   * profile = 2 only records the events and reads them after the solve, so
   * launches keep their normal pacing (streaming SDSN passes are then timed
   * per enqueued chunk). */
  int gemm_launches;     /* GEMM launches (two per outer iteration)                    */
  int sdsn_launches;     /* SDSN launches that did work (on-chip: one per projection)  */
  double ms_gemm;        /* GEMM 1 + GEMM 2                                            */
  double ms_sdsn;        /* SDSN passes (excluding the final gamma check)              */
  double ms_stats;       /* tile statistics of X that start each SDSN call            */
  double ms_update;      /* N update + delta                                           */
  int stalled;           /* 1 if the delta-stall rule (fram_options.stall_iters) stopped
                            the loop                                                   */
  double ms_discretize;  /* (profile 1 or 2) Algorithm 1 step 10 on the device: row
                            argmax, column minima and the exact assignment           */
  int sdsn_onchip;       /* projections run by the on-chip SDSN launch                 */
  int sdsn_fallbacks;    /* on-chip launches that did not complete, and whose
                            projection therefore streamed (same result): either not
                            all workgroups became resident within the roll-call bound
                            (compute units held by other work), or a pass barrier
                            waited past its bound (e.g. the launch's hardware queue
                            was preempted) and the launch was abandoned before it
                            wrote anything                                          */
} fram_stats;

typedef struct {
  fram_precision prec;   /* GEMM input type; default FRAM_FP32                         */
  double alpha;          /* step size of Algorithm 1 step 7; default 0.95 (Sec. 7)     */
  double gamma_tol;      /* SDSN stop: gamma <= gamma_tol; default 1e-6                */
  int sdsn_max;          /* SDSN pass cap per call; default 1000                       */
  int tile;              /* 0 = automatic, else 64 / 128 / 256                          */
  int profile;           /* 0 = off; 1 = time each launch alone; 2 = time launches
                            without serialising them (see fram_stats)                 */
  int stable_iters;      /* w > 0: also stop once the row argmax of N has been the same
                            permutation for w consecutive iterations (a second stop
                            rule beside delta <= tol, for precisions whose delta
                            levels off above tol); 0 = off (default)                 */
  int sdsn_mode;         /* 0 = automatic: on-chip whenever the grid fits the device
                            (n up to ~4400) and the matrix is more than one tile, else
                            streaming; 1 = one streaming launch per SDSN pass; 2 =
                            on-chip: all passes of a projection (and, in solves, the N
                            update of Algorithm 1 step 7) in one launch with the
                            iterate held in registers (FRAM_EINVAL if the device cannot
                            hold it).  On-chip launches of all contexts and streams
                            of the process are admitted only while the grids that may
                            still run fit on the device together; one whose workgroups
                            cannot all be resident within the roll-call bound, or
                            whose pass barrier waits past its bound, writes nothing
                            and that projection streams instead
                            (fram_stats.sdsn_fallbacks).  Both modes give the same
                            iterates bit for bit.                                    */
  int stall_iters;       /* w > 0: also stop once delta has stalled at the precision's
                            floor: after delta <= stall_delta, w consecutive iterations
                            without a new smallest delta; 0 = off (default)            */
  double stall_delta;    /* delta below which stalls are counted; default 1e-3          */
  int variant;           /* 0 = FRAM (default); 1 = DSPFP, the baseline iteration FRAM
                            modifies (Sec. 4, eq. iter.DSPFP): the same outer loop with
                            the plain alternating doubly stochastic projection of the
                            unscaled gradient (no theta, no division by max X) for a
                            fixed dsn_iters passes, stopping on DSPFP's own criterion
                            max |N/max N - N_prev/max N_prev| <= tol (App. B.2), which
                            fram_stats.delta then reports.  Solve entry points only;
                            not with node similarities (FRAM_EINVAL).               */
  int dsn_iters;         /* DSPFP projection passes per outer iteration; default 30     */
  int many_workers;      /* fram_solve_many: pairs solved at the same time, each on a
                            worker context with its own stream (one host thread each);
                            1..32, default 16.  Streams share the process's hardware
                            queues (HIP's GPU_MAX_HW_QUEUES, read when HIP starts):
                            measured on 512 pairs of n in [20, 300], 16 workers give
                            115 pairs/s with 4 queues and 216 with 16              */
  const float* N0;       /* warm start of Algorithm 1 step 1: NULL (default) starts from
                            N = 0; else n*n floats, row-major, finite, used as N^(0)
                            (host memory for the host entry points, device memory with
                            leading dimension n for the _dev ones).  A solve of a + b
                            fixed iterations (tol = 0) equals, bit for bit, a solve of a
                            iterations whose N_out is passed as N0 to a solve of b: the
                            iterate is the whole state of the loop (the stop-rule
                            counters of stall_iters / stable_iters restart with the
                            call).  Single-pair solves only (fram_solve_many: EINVAL). */
  float* N_out;          /* NULL (default) or n*n floats (same memory kind as N0): the
                            final iterate N, before discretisation (not written for
                            n = 1, which needs no iteration)                          */
  int onchip_roll_us;    /* bound on the roll call of an on-chip launch (all workgroups
                            resident), microseconds; 0 = default (10 000)            */
  int onchip_barrier_us; /* bound on each pass barrier wait of an on-chip launch,
                            microseconds; 0 = default (20 000).  A pass takes a few
                            microseconds; the bound only ends a launch that has
                            stopped progressing.  Tiny bounds force the fallbacks
                            (same results), e.g. in tests                            */
} fram_options;

/* Sizes of fram_options and fram_stats as compiled into the library, for
 * bindings that mirror the structs. */
void fram_struct_sizes(size_t* options_bytes, size_t* stats_bytes);

typedef struct fram_ctx fram_ctx;

/* Fill *opt with the defaults listed above. */
void fram_default_options(fram_options* opt);

/* Create a context bound to HIP device `device`.  hbm_budget_bytes caps the
 * device workspace the context may hold (0 = no cap beyond device memory).
 * No HIP call is made here: the device is initialised on first use.
 * Returns FRAM_EINVAL if out is NULL or device < 0. */
fram_status fram_create(fram_ctx** out, int device, size_t hbm_budget_bytes);

/* Release the context and its device workspace.  NULL is accepted. */
void fram_destroy(fram_ctx* ctx);

/* Bytes of device workspace a solve of size n at precision prec needs; used by
 * the budget check and by admission control.  Pure host arithmetic. */
size_t fram_workspace_bytes(int n, fram_precision prec, int tile);

/* Autotune table for the automatic tile choice (fram_options.tile == 0): the
 * square tile edge of the SDSN passes and GEMMs of a solve or projection of
 * size n.  Bucket k covers n_max[k-1] < n <= n_max[k] (n_max strictly
 * increasing, >= 1) and selects tile[k] (64, 128 or 256); sizes above the
 * last bucket keep the built-in rule (one tile up to n = 128: 64 for
 * n <= 64, else 128; above, the largest tile whose grid has at least 200
 * tiles, else 64).  The table is copied; it is shared by every
 * context of the process and also governs fram_workspace_bytes(.., 0).
 * count == 0 clears it.  At most 64 buckets.  Returns FRAM_EINVAL (table
 * unchanged) on a count out of range, a NULL array with count > 0, an
 * n_max that is not strictly increasing and positive, or a tile not in
 * {64, 128, 256}.  Calls that race with solves being planned on other
 * threads are safe; each solve uses the table as it was when it started.
 * Results can differ in the last bits between tile edges (the FP64 partial
 * sums of the SDSN pass are combined per tile). */
fram_status fram_set_tile_table(const int* n_max, const int* tile, int count);

/* Tile edge the automatic choice gives for size n (table, else built-in
 * rule); 0 when n is outside [1, FRAM_MAX_N].  Pure host arithmetic. */
int fram_auto_tile(int n);

/* FRAM, Algorithm 1 (with Algorithm 2 as its projection), on host inputs.
 *   A, B      host, n*n doubles, row-major; symmetric, finite, >= 0 (Sec. 3).
 *   n         >= 1.  n == 1 returns perm {0}.
 *   lambda    theta of Theorem 1, > 0 (the paper uses 2 for dense graphs and
 *             10 for sparse ones, Sec. 7).
 *   iters     >= 1, cap on outer iterations.
 *   tol       >= 0, delta threshold; the loop is a do-while and stops when
 *             delta <= tol (tol = 0 runs exactly `iters` iterations).
 *   perm_out  host, n int32 (written).   objective_out  host, 1 double (written).
 * Uses fram_default_options (FP32 GEMMs). */
fram_status fram_solve(fram_ctx* ctx, const double* A, const double* B, int n,
                       double lambda, int iters, double tol,
                       int32_t* perm_out, double* objective_out);

/* As fram_solve with explicit options (NULL = defaults) and stats (may be NULL). */
fram_status fram_solve_ex(fram_ctx* ctx, const double* A, const double* B, int n,
                          double lambda, int iters, double tol, const fram_options* opt,
                          int32_t* perm_out, double* objective_out, fram_stats* stats);

/* As fram_solve_ex with A and B already in device memory (dA, dB: n*n doubles,
 * row-major, leading dimension n), work ordered on `stream` (a hipStream_t, or
 * NULL for the context's own stream).  Symmetry/sign/finiteness of the device
 * inputs are checked by a device kernel before the solve (FRAM_EINVAL).
 * perm_out and objective_out are host pointers. */
fram_status fram_solve_dev(fram_ctx* ctx, const double* dA, const double* dB, int n,
                           double lambda, int iters, double tol, const fram_options* opt,
                           int32_t* perm_out, double* objective_out, fram_stats* stats,
                           void* stream);

/* SDSN, Algorithm 2, alone: X_out = SDSN(K, theta).
 *   K       host, n*n floats, row-major (any real values).
 *   lambda  theta > 0.
 *   X_out   host, n*n floats (written): nonnegative, row and column sums within
 *           n*gamma_tol of 1 unless the pass cap was hit.
 * X^(0) = (theta/2) K / max(K); a K with max <= 0 starts from the zero matrix,
 * giving 11^T/n.  At least one pass is made. */
fram_status fram_sdsn_project(fram_ctx* ctx, const float* K, int n, double lambda,
                              float* X_out);

/* As fram_sdsn_project with options (gamma_tol, sdsn_max) and stats
 * (sdsn_passes, gamma, sdsn_capped). */
fram_status fram_sdsn_project_ex(fram_ctx* ctx, const float* K, int n, double lambda,
                                 const fram_options* opt, float* X_out, fram_stats* stats);

/* Device-memory SDSN: dK and dX are device pointers (n*n floats, leading
 * dimensions ldk, ldx >= n); dX may equal dK. */
fram_status fram_sdsn_project_dev(fram_ctx* ctx, const float* dK, int ldk, int n,
                                  double lambda, const fram_options* opt, float* dX,
                                  int ldx, fram_stats* stats, void* stream);

/* Largest n fram_sdsn_project_noalloc takes. */
#define FRAM_NOALLOC_MAX_N 1024

/* fram_sdsn_project_dev for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no context, and no allocation of any kind -- the working memory
 * (padded iterate, tile partials, state; at most 6 MiB) is a file-scope device
 * array of the library, one per GPU, held until the process ends.
 *   dK, dX   device, n x n floats with leading dimensions ldk, ldx >= n
 *            (dX may equal dK); n <= FRAM_NOALLOC_MAX_N (else FRAM_EINVAL).
 *   opt      NULL = defaults; gamma_tol, sdsn_max and tile (0, 64 or 128) are
 *            used; sdsn_mode 2 (on-chip) is FRAM_EINVAL: the streaming passes
 *            always run, the same kernels as fram_sdsn_project_dev's
 *            streaming mode, so X is the same bit for bit.
 *   stats    NULL or written (sdsn_passes, gamma, sdsn_capped, gemm_tile).
 *   stream   a hipStream_t (NULL = the default stream); the call returns after
 *            the stream has finished the projection.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (each call clears what must start at zero): calls that overlap
 * on one GPU, from several threads or streams, race and must be serialised by
 * the caller. */
fram_status fram_sdsn_project_noalloc(const float* dK, int ldk, int n, double lambda,
                                      const fram_options* opt, float* dX, int ldx,
                                      fram_stats* stats, void* stream);

/* Gradient of eq. (3) alone, for kernel checks: X = A * N * B computed as
 * W = B N^T (GEMM 1) and X = A W^T (GEMM 2) with inputs rounded to `prec`
 * and FP32 accumulation; W is held in `prec`.  All pointers are host, n*n,
 * row-major; A and B must be symmetric (B^T = B is used). */
fram_status fram_gradient(fram_ctx* ctx, const float* A, const float* N, const float* B,
                          int n, fram_precision prec, float* X_out);

/* FRAM on attributed graphs: the node term of eq. (1), lambda <N, K> with
 * K = F F~^T (Sec. 3), enters every gradient of eq. (3) / Algorithm 1 step 5:
 * X = A N A~ + node_weight K.  Algorithm 1 steps 2-3 scale K with the edges
 * (here: by 1 / (max A max A~), which differs from the paper's c-scaling only
 * by a positive factor common to both terms, which SDSN divides out).
 *   K            n*n doubles, row-major, finite (any sign, need not be
 *                symmetric); host for _ex, device for _dev.
 *   node_weight  the lambda of eq. (1) (the paper uses 1); finite.
 *   objective_out = 2 Phi(M) = sum_{k,l} A_kl B_{s(k)s(l)} + 2 node_weight
 *                sum_k K[k, s(k)], in FP64 on the unscaled inputs.
 * n = n~ as in the paper's formulation (Sec. 3).  Everything else as
 * fram_solve_ex / fram_solve_dev (lambda there is the SDSN strength theta). */
fram_status fram_solve_attr_ex(fram_ctx* ctx, const double* A, const double* B, const double* K,
                               int n, double node_weight, double lambda, int iters, double tol,
                               const fram_options* opt, int32_t* perm_out, double* objective_out,
                               fram_stats* stats);

fram_status fram_solve_attr_dev(fram_ctx* ctx, const double* dA, const double* dB,
                                const double* dK, int n, double node_weight, double lambda,
                                int iters, double tol, const fram_options* opt, int32_t* perm_out,
                                double* objective_out, fram_stats* stats, void* stream);

/* Exact linear assignment of Algorithm 1 step 10 / eq. (2), the discretisation
 * the paper does with the Hungarian method (Sec. 6): perm_out maximises
 * sum_i W[i, perm_out[i]], i.e. it is the permutation P minimising ||P - W||_F.
 * Runs on the device in three phases: row maxima as the starting duals and
 * column minima of the reduced costs as the starting prices; bids of the free
 * rows (Jonker-Volgenant augmenting row reduction: for n < 1024 two
 * sequential passes, at most 4 * free + n / 2 bids; from n = 1024 parallel
 * rounds in which every free row bids at once and each column goes to its
 * largest bid, until no row is left or 8 rounds bring no progress); then one
 * shortest augmenting path (with row and column potentials) per row still
 * free.  When the row argmax is already a
 * permutation it is returned as is.  Ties go to the lowest column.  The
 * solvers use the same device code for their final step.
 *   W        host, n*n floats, row-major, finite (else FRAM_EINVAL).
 *   perm_out host, n int32 (written).
 * fram_last_stats().lap_paths reports the rows the row argmax left free. */
fram_status fram_assign(fram_ctx* ctx, const float* W, int n, int32_t* perm_out);

/* Same on device memory: dW n x n floats with leading dimension ldw >= n,
 * dperm n int32 (written), on `stream` (a hipStream_t; NULL = the context's
 * stream).  Returns after the stream has finished the assignment.  A matrix
 * with non-finite entries gives FRAM_ENUMERIC and dperm filled with -1. */
fram_status fram_assign_dev(fram_ctx* ctx, const float* dW, int ldw, int n, int32_t* dperm,
                            void* stream);

/* Many independent pairs (uneven n), each solved as by fram_solve_ex.
 *   count        >= 1 pairs; A[i], B[i] host n[i]*n[i] doubles.
 *   perm_out[i]  host, n[i] int32 (written); objective_out host, count doubles.
 *   opt          NULL = defaults; opt->N0 / opt->N_out must be NULL.
 *   stats        NULL or count entries.
 * Pairs whose matrix is a single tile (2 <= n <= 256; edge 64, 128 or 256)
 * are solved in lockstep on a group context of ctx: each outer iteration of
 * Algorithm 1 is one launch per kernel for all pairs still running (the two
 * GEMMs, the whole SDSN projection of each pair in one workgroup, the N
 * update and delta) and one copy of all their states to the host, where
 * every pair's stop rules are applied; a pair leaves the group when it stops.
 * A grouped pair's result equals, bit for bit, solving it alone with
 * opt->tile set to its edge (for n <= 128 that is the default layout).  Pairs
 * are grouped only with the FRAM variant, stable_iters = 0, profile = 0,
 * sdsn_mode 0 or 1 and opt->tile 0 or the pair's edge.  The other pairs are
 * spread over worker contexts of ctx (opt->many_workers of them, each with its
 * own stream, workspace and host thread), concurrently with the group, every
 * pair running the single-pair solve on its worker, so its result is the
 * same as when it is solved alone.  The first error stops the call and is
 * returned (later pairs are then left unwritten). */
fram_status fram_solve_many(fram_ctx* ctx, int count, const double* const* A,
                            const double* const* B, const int* n, double lambda, int iters,
                            double tol, int32_t* const* perm_out, double* objective_out);

fram_status fram_solve_many_ex(fram_ctx* ctx, int count, const double* const* A,
                               const double* const* B, const int* n, double lambda,
                               int iters, double tol, const fram_options* opt,
                               int32_t* const* perm_out, double* objective_out,
                               fram_stats* stats);

/* Device memory the context holds between calls: its workspace (which only
 * grows, to the largest problem solved so far), that of its fram_solve_many
 * workers and group, and its small fixed buffers.  Pure host bookkeeping. */
size_t fram_resident_bytes(const fram_ctx* ctx);

/* Release the workspace of the context, its workers and its group (after
 * waiting for their streams); the next call allocates again.  For admission control that
 * must bound the memory held by idle contexts.  NULL is accepted. */
fram_status fram_trim(fram_ctx* ctx);

/* Stats of the last call on this context. */
fram_status fram_last_stats(const fram_ctx* ctx, fram_stats* out);

/* Static text for a status code. */
const char* fram_status_str(fram_status s);

/* Text of the last error on this context ("" if none). */
const char* fram_last_error(const fram_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* FRAM_H */
