/* farpca.h - C-ABI of the MI355X (gfx950) implementation of the accelerated
 * farPCA hot path: the blocked, adaptive randomized QB / PCA loop of
 * Algorithm 1 (farPCA, Section 2.1) with the sparse test matrices of
 * Definitions 2.1-2.4 (farPCASB = Algorithm 2; farPCASS, farPCASG, farPCAB of
 * Sections 3.2 and 5) of Jiang, Fu, Xu, "Accelerating Randomized Algorithms for
 * Low-Rank Matrix Approximation" (arXiv 2506.03859).
 *
 * Conventions
 *  - All matrices are row-major FP32 unless stated.  A is m x n with leading
 *    dimension lda >= n (elements).  Any m, n >= 1 is accepted (m < n too).
 *    The whole m x lda array must be readable: the kernels may read a row's
 *    padding between n and lda (never using its values).  Rows of 16 bytes
 *    (lda a multiple of 4 for FP32, of 8 for BF16) on a 16-byte-aligned base
 *    take the vector load paths; other layouts take slower element loads.
 *  - Pointers named d* are device pointers (global memory of the current HIP
 *    device), owned by the caller.  The library allocates no device memory
 *    while it runs: scratch buffers live in the caller's workspace, in a static
 *    device array (farpca_run_static) or in a server's pool (allocated once by
 *    farpca_server_create).
 *  - `stream` is a hipStream_t passed as void*; all device work is enqueued on
 *    it.  farpca_run is host-synchronous: it reads the error indicator after
 *    every block (one 8-byte device-to-host copy) and returns after the final
 *    decomposition has been written.
 *  - Errors are returned as negative status codes; no exception crosses the
 *    ABI.  On error the output buffers are unspecified.
 *  - A plan holds host-side state only.  One plan must not be used by two
 *    threads at once; distinct plans may run concurrently on distinct streams
 *    with distinct workspaces.
 */
#ifndef FARPCA_H_
#define FARPCA_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define FARPCA_OK 0              /* fixed precision: E < tol^2 ||A||_F^2 reached; fixed rank: done */
#define FARPCA_NOT_CONVERGED 1   /* block cap reached first; outputs valid at l = blocks * b       */
#define FARPCA_E_INVALID (-1)    /* invalid parameter                                              */
#define FARPCA_E_NOMEM (-2)      /* workspace smaller than farpca_plan reported                    */
#define FARPCA_E_DEVICE (-3)     /* a HIP call failed                                              */
#define FARPCA_E_NONFINITE (-4)  /* A holds NaN or Inf                                             */

/* test matrices (Definitions 2.1-2.4) */
#define FARPCA_GAUSSIAN 0         /* dense standard Gaussian G_j (farPCA, Algorithm 1)           */
#define FARPCA_STD_BERNOULLI 1    /* standardized Bernoulli (B-p)/sqrt(p(1-p)) (Def. 2.3, Alg. 2) */
#define FARPCA_SPARSE_SIGN 2      /* sparse sign (Def. 2.2; zeta > 0: zeta nonzeros per row)     */
#define FARPCA_SPARSE_GAUSSIAN 3  /* sparse Gaussian B o G / sqrt(p) (Def. 2.4)                  */
#define FARPCA_BERNOULLI 4        /* plain 0/1 Bernoulli (Def. 2.1, farPCAB of Section 5)        */

#define FARPCA_DTYPE_F32 0
/* Precision form: A stored as BF16 (uint16 bit patterns, the caller's rounding,
 * normally round-to-nearest-even from FP32).  The A-passes run on the BF16
 * matrix cores with FP32 accumulation; the FP32 vectors they multiply are
 * split exactly into three BF16 terms, so every product A_ij x_j is exact and
 * the results equal those of the FP32 path on the BF16-valued matrix up to
 * FP32 accumulation order.  Everything else (sketch sums, Grams, Cholesky,
 * indicator, eigensolver) is unchanged.  The method's accuracy is then bounded
 * by the storage error ||A - A_bf16||_F / ||A||_F (unit roundoff 2^-8; about 2e-3 for generic data). */
#define FARPCA_DTYPE_BF16 1

/* Storage order of A */
#define FARPCA_LAYOUT_ROW 0  /* row-major: element (i, k) at dA[i * lda + k], lda >= n             */
/* Column-major (A^T row-major): element (i, k) at dA[k * lda + i], lda >= m; FP32 only.  The
 * sparse sketch then gathers whole columns of A: it reads the columns that Omega_j touches,
 * nnz(Omega_j) m elements rather than m n (Section 3, the cost of A B_j), which is the layout the
 * paper's sparse test matrices with p near 1e-3 pay off in.  The sketch reads each column of A
 * once per nonzero in its row of Omega_j, so this layout suits few nonzeros per row (a sparse
 * sign matrix with zeta = 8 reads A 8 times over).  The A-passes and the setup run as the
 * transposed products / column sums of the stored matrix; the results equal the row-major
 * path's up to FP32 accumulation order. */
#define FARPCA_LAYOUT_COL 1

typedef struct farpca_params {
  int64_t m, n, lda;   /* A is m x n, leading dimension lda (>= n row-major, >= m column-major) */
  int32_t a_dtype;     /* FARPCA_DTYPE_F32 or FARPCA_DTYPE_BF16                              */
  int32_t sketch;      /* FARPCA_GAUSSIAN ... FARPCA_BERNOULLI                               */
  double tol;          /* relative Frobenius tolerance eps > 0 (fixed precision, Section 5.2):
                          stop once E < eps^2 ||A||_F^2 (strict); ignored when rank > 0     */
  int64_t rank;        /* k > 0: fixed-rank use (Section 5.1), blocks until l = j b >= k     */
  int32_t block;       /* b in [1, 64]; 0 = min(max(20, floor(min(m,n)/100)), 50) (5.2/5.4)  */
  int32_t power;       /* P >= 0 power steps per block (shift active for P > 2)              */
  int64_t max_blocks;  /* 0 = ceil(min(m,n) / (2 b)) (Section 5.2); l is also capped at min(m,n) */
  double sketch_p;     /* Bernoulli / density p in (0,1); 0 = p1 = max(1e-3, ln n/n) for
                          FARPCA_STD_BERNOULLI, p2 = max(1e-3, 10/n) otherwise (Section 5;
                          n = rows of Omega_j: about ln n or 10 nonzeros per column)      */
  int32_t sketch_zeta; /* FARPCA_SPARSE_SIGN: zeta in [1, b] nonzeros +-1/sqrt(zeta) per row
                          of Omega_j; 0 = i.i.d. entries of Definition 2.2                   */
  int32_t a_layout;    /* FARPCA_LAYOUT_ROW (0) or FARPCA_LAYOUT_COL                         */
  uint64_t seed;       /* key of the counter-based generator (Philox4x64-10)                 */
} farpca_params;

typedef struct farpca_info {
  int64_t rank_l;        /* basis size l = blocks * b                                         */
  int64_t rank_out;      /* columns written to U, S, V (k in fixed-rank use, else l)          */
  int32_t blocks;        /* blocks computed                                                   */
  int32_t status;        /* FARPCA_OK or FARPCA_NOT_CONVERGED                                 */
  double norm_a2;        /* ||A||_F^2 (FP64)                                                  */
  double err_indicator;  /* E = ||A||_F^2 - ||Q^T A||_F^2 after the last block (FP64)         */
  int32_t eig_sweeps;    /* Jacobi sweeps of the final eigendecomposition                     */
  int32_t dropped;       /* nonzero if a block direction was dropped as numerically dependent
                            (its column of U, V is zero and its singular value 0)     */
  int64_t rank_trunc;    /* post-processing for the fixed-precision problem (Section 5.4, after
                            Hallman's block method): the smallest r such that the first r
                            singular triplets still meet the tolerance,
                            E + sum_{i >= r} S_i^2 < tol^2 ||A||_F^2 (S descending; the rank-r
                            truncation error, since A - Q Q^T A is orthogonal to range(Q)).
                            rank_out when the run did not converge or in fixed-rank use.  */
  int32_t eig_converged; /* 1 if the final eigensolver met its off-diagonal test
                            (|k_pq| <= 1e-7 sqrt(k_pp k_qq) after the sweeps, so V is
                            orthonormal to that level, or stalled below 1e-11 of it);
                            0 if it stopped at its cap of FARPCA_EIG_MAX_SWEEPS sweeps
                            (U S V^T = Q Q^T A still holds)                          */
  int32_t reserved1;
} farpca_info;

typedef struct farpca_plan_s farpca_plan_t;

/* Validate parameters and size the work.  On success *out holds a new plan,
 * *l_max the largest basis size the run can reach (U, V need l_max columns,
 * S l_max entries) and *workspace_bytes the device workspace farpca_run needs.
 * Returns FARPCA_OK or FARPCA_E_INVALID. */
int farpca_plan(const farpca_params *params, farpca_plan_t **out, int64_t *l_max,
                size_t *workspace_bytes);

/* Run the method (Algorithms 1/2 with the steps of the plan).
 *  dA     device, m x n FP32 or BF16 (a_dtype; lda elements), read only
 *  dWork  device workspace, >= workspace_bytes, 256-byte aligned, contents ignored
 *  dU     device, m x l_max FP32 (leading dimension l_max): left singular vectors
 *  dS     device, l_max FP64: singular values, descending
 *  dV     device, n x l_max FP32 (leading dimension l_max): right singular vectors
 *  info   host, filled on return (may be NULL)
 *  dEhist device, l_max / b FP64 or NULL: E after every block
 * Only the first info->rank_out columns / entries of U, S, V are written. */
int farpca_run(farpca_plan_t *plan, const void *dA, void *dWork, size_t work_bytes, void *dU,
               double *dS, void *dV, farpca_info *info, double *dEhist, void *stream);

/* The same run in three calls, for a caller that schedules solves block by block
 * (for instance one block of each of several requests in turn on one stream).
 * farpca_run is exactly farpca_begin, farpca_step until it returns 0, farpca_finish:
 * the same kernels in the same order, so the results are bitwise the same.
 *  farpca_begin   step a0 (||A||_F^2, finiteness, the standardized Bernoulli row
 *                 sums); A, dWork and dEhist (may be NULL) must stay valid and
 *                 untouched until farpca_finish returns.  Returns FARPCA_OK,
 *                 FARPCA_E_NONFINITE, FARPCA_E_NOMEM or FARPCA_E_INVALID.
 *  farpca_step    one block of Algorithm 1/2 (test matrix, sketch, power steps,
 *                 basis extension, indicator update) and the stop test, which reads
 *                 E back (host-synchronous).  Returns 1 if another block is needed,
 *                 0 once the tolerance, the rank or the block cap is reached (also on
 *                 calls after that), FARPCA_E_INVALID before farpca_begin.
 *  farpca_finish  the final decomposition (U, S, V as farpca_run) and info; returns
 *                 FARPCA_OK or FARPCA_NOT_CONVERGED, FARPCA_E_INVALID if no block ran.
 * The run state lives in the plan (host side): one run per plan at a time. */
int farpca_begin(farpca_plan_t *plan, const void *dA, void *dWork, size_t work_bytes,
                 double *dEhist, void *stream);
int farpca_step(farpca_plan_t *plan, void *stream);
/* farpca_step in two halves, for a scheduler that keeps blocks of many solves
 * in flight from one host thread:
 *  farpca_step_async  enqueues the next block on `stream` (the same kernels as
 *                     farpca_step) and an asynchronous read-back of E; returns 1
 *                     when a block was enqueued, 0 if the run needs no further
 *                     block, FARPCA_E_INVALID before farpca_begin or while a
 *                     block is still pending (poll it first);
 *  farpca_step_poll   examines the pending block's E once it is complete:
 *                     returns 2 if it is still running (wait = 0; wait != 0
 *                     blocks until it completes), else as farpca_step (1: another
 *                     block is needed, 0: stop).
 * farpca_step is farpca_step_async followed by farpca_step_poll(plan, 1).  The
 * read-back uses a few bytes of pinned host memory and an event held by the
 * plan (created on the first block, released by farpca_free). */
int farpca_step_async(farpca_plan_t *plan, void *stream);
int farpca_step_poll(farpca_plan_t *plan, int wait);

/* Block-granular memory, for callers that grow a solve's memory with its basis
 * (a serving pool).  The workspace of farpca_run has two parts: the loop part
 * (everything the blocks need; Q and C^T with room for every block) and the
 * final part (step a10, sized for l_max).  Instead, a run may start on a loop
 * part with room for cap_blocks blocks, move to a larger one between blocks,
 * and take the final part, sized for the l it reached, only at the end:
 *  farpca_loop_bytes   size of the loop part with room for cap_blocks blocks
 *                      (1 <= cap_blocks <= l_max / b), 0 if invalid;
 *  farpca_begin_loop   farpca_begin on such a loop part (device, 256-byte aligned);
 *  farpca_step_async / farpca_step / farpca_step_poll as above; farpca_step_async
 *                      returns FARPCA_E_NOMEM when the next block needs more room;
 *  farpca_grow         between blocks (no block pending): moves the run to a new loop
 *                      part with room for cap_blocks >= the current capacity: enqueues
 *                      on `stream` the copies of what the loop carries (Q and C^T, the
 *                      scalars, the row sums, the E history when it is internal).  The
 *                      old loop part must stay untouched until those copies have run
 *                      (stream order; e.g. release it after an event on `stream`);
 *  farpca_final_bytes  once the block loop has ended: size of the final part for the
 *                      reached l (outputs not included);
 *  farpca_finish_final farpca_finish with the final part at dFinal (device, 256-byte
 *                      aligned, farpca_final_bytes bytes) and outputs U (m x ldu), S,
 *                      V (n x ldv), ldu, ldv >= info.rank_out.  The loop part and the
 *                      final part may be released once it returns.
 * The kernels and their order are those of farpca_run, so the results are bitwise
 * the same (only the leading dimensions of Q, C^T, U and V differ). */
size_t farpca_loop_bytes(farpca_plan_t *plan, int64_t cap_blocks);
int farpca_begin_loop(farpca_plan_t *plan, const void *dA, void *dLoop, size_t bytes,
                      int64_t cap_blocks, double *dEhist, void *stream);
int farpca_grow(farpca_plan_t *plan, void *dLoop, size_t bytes, int64_t cap_blocks, void *stream);
size_t farpca_final_bytes(farpca_plan_t *plan);
int farpca_finish_final(farpca_plan_t *plan, void *dFinal, size_t bytes, void *dU, int64_t ldu,
                        double *dS, void *dV, int64_t ldv, farpca_info *info, void *stream);
int farpca_finish(farpca_plan_t *plan, void *dU, double *dS, void *dV, farpca_info *info,
                  void *stream);

/* farpca_run for callers that cannot allocate device memory (code that must not
 * call hipMalloc: tight serving loops, harnesses that forbid allocation).  The
 * workspace is a device array of FARPCA_STATIC_SCRATCH_BYTES inside the library,
 * one per GPU, held from the library's load until the process ends; the call
 * itself allocates nothing (the caller still passes A and the outputs, as for
 * farpca_run, and the same kernels run in the same order, so the results are
 * bitwise those of farpca_run).  Returns FARPCA_E_NOMEM when the plan's
 * workspace_bytes exceeds FARPCA_STATIC_SCRATCH_BYTES; otherwise as farpca_run.
 * All calls on one GPU share that GPU's array: calls that overlap on one GPU
 * (from several threads or streams) race and must be serialised by the caller. */
#define FARPCA_STATIC_SCRATCH_BYTES (64u << 20)
int farpca_run_static(farpca_plan_t *plan, const void *dA, void *dU, double *dS, void *dV,
                      farpca_info *info, double *dEhist, void *stream);

void farpca_free(farpca_plan_t *plan);
const char *farpca_status_str(int status);

/* ---- step entry points (same kernels as farpca_run; used by the parity tests)
 * farpca_omega: test matrix Omega_j of block j (blocks count from 0).
 *   dMask  device n x uint64: bit c set iff entry (r, c) is nonzero
 *   dNeg   device n x uint64: bit c set iff entry (r, c) is negative
 *   dDense device n x 64 FP32: the matrix the sketch multiplies by, i.e. the
 *          definition's values (standardized Bernoulli: B_j - p, the unscaled
 *          form of Algorithm 2); columns >= b are zero.
 * farpca_sketch: dS (m x 64 FP32, columns >= b zero) = A * dDense, computed by
 *   the sparse gather kernel (dense GEMM for FARPCA_GAUSSIAN); standardized
 *   Bernoulli: A B_j - z with z = A (p 1_n) (Section 3.1).  dA in the plan's
 *   storage (a_dtype, a_layout): column-major A is gathered by columns.
 * Both need the workspace of farpca_plan. */
int farpca_omega(farpca_plan_t *plan, int64_t block_j, void *dWork, size_t work_bytes,
                 uint64_t *dMask, uint64_t *dNeg, float *dDense, void *stream);
int farpca_sketch(farpca_plan_t *plan, const void *dA, int64_t block_j, void *dWork,
                  size_t work_bytes, float *dS, void *stream);

/* FP32 matrix-core products used by the loop (N <= 64, C row-major ldc):
 *  farpca_gemm_nn: C[M x N] = A[M x K] X[K x N]       (A lda, X ldx)
 *  farpca_gemm_tn: C[M x N] = A^T Y, A is K x M       (A lda, Y ldy)
 * dPart: device scratch of farpca_gemm_scratch_bytes(M) bytes (split-K partials). */
size_t farpca_gemm_scratch_bytes(int64_t M);
int farpca_gemm_nn(const float *dA, int64_t lda, const float *dX, int64_t ldx, float *dC,
                   int64_t ldc, int64_t M, int64_t N, int64_t K, float *dPart, void *stream);
int farpca_gemm_tn(const float *dA, int64_t lda, const float *dY, int64_t ldy, float *dC,
                   int64_t ldc, int64_t M, int64_t N, int64_t K, float *dPart, void *stream);

/* The same two products with A in BF16 (bit patterns, as for FARPCA_DTYPE_BF16):
 * BF16 matrix cores, the FP32 operand X / Y split exactly into three BF16
 * terms, FP32 accumulation.  dScratch: device, farpca_gemm_bf16_scratch_bytes(M, K)
 * bytes, 256-byte aligned (split-K partials and the transposed operand).  The
 * whole row-major array of A (rows x lda) must be readable (row padding may be
 * read, never used). */
size_t farpca_gemm_bf16_scratch_bytes(int64_t M, int64_t K);
int farpca_gemm_bf16_nn(const uint16_t *dA, int64_t lda, const float *dX, int64_t ldx, float *dC,
                        int64_t ldc, int64_t M, int64_t N, int64_t K, void *dScratch, void *stream);
int farpca_gemm_bf16_tn(const uint16_t *dA, int64_t lda, const float *dY, int64_t ldy, float *dC,
                        int64_t ldc, int64_t M, int64_t N, int64_t K, void *dScratch, void *stream);

/* The FP32 products on the BF16 matrix cores (the dense A-passes of Algorithms
 * 1 and 2 with A in FP32): both operands are split exactly into three BF16
 * terms (rounding to nearest; each difference is exact in FP32) and six of
 * the nine term products are accumulated in FP32 (hi hi, hi mid, mid hi, mid
 * mid, hi lo, lo hi).  The three left out are below 2^-23 |a x| per product
 * together and of either sign (about one FP32 rounding of the product), so
 * the result carries FP32-level rounding, not BF16's.  In the TN product each
 * 32-deep slice's products are summed from zero and added to the running sum
 * in FP32 by the vector unit (no bias in sums of squares of its columns: it
 * forms C_j^T = A^T Q_j of the indicator).  Same arguments, scratch
 * (farpca_gemm_bf16_scratch_bytes) and readability rule as the BF16 products,
 * with A FP32. */
int farpca_gemm_f32s_nn(const float *dA, int64_t lda, const float *dX, int64_t ldx, float *dC,
                        int64_t ldc, int64_t M, int64_t N, int64_t K, void *dScratch, void *stream);
int farpca_gemm_f32s_tn(const float *dA, int64_t lda, const float *dY, int64_t ldy, float *dC,
                        int64_t ldc, int64_t M, int64_t N, int64_t K, void *dScratch, void *stream);

/* FP64 symmetric eigendecomposition (block Jacobi) of K (l x l, row-major):
 * dW (l) descending, dV (l x l) eigenvectors in columns.  dWork holds
 * farpca_eig_scratch_bytes(l) bytes.  The sweeps stop once every off-diagonal
 * entry of V^T K V meets |k_pq| <= rel sqrt(|k_pp k_qq|) (rel <= 0: 1e-14; the
 * final step of farpca_run uses 1e-7) or |k_pq| <= 4e-15 max|k_ii| (the FP64
 * rounding of the largest entry), or once two sweeps in a row halve neither the
 * largest ratio |k_pq| / sqrt(|k_pp k_qq|) nor the largest |k_pq| of the failing
 * entries while the ratio is below 1e-11 or the entry below 1e-12 max|k_ii|
 * (the rounding level of the rotations).  Returns the sweep count (>= 0) or an error;
 * *converged (host, may be NULL) is 1 if that happened within
 * FARPCA_EIG_MAX_SWEEPS sweeps, else 0. */
#define FARPCA_EIG_MAX_SWEEPS 40
size_t farpca_eig_scratch_bytes(int64_t l);
int farpca_eig(const double *dK, int64_t l, double *dW, double *dV, void *dWork, double rel,
               int *converged, void *stream);

/* ---- serving: continuous batching of independent solves on one GPU
 * A server owns one device pool of pool_bytes (allocated by
 * farpca_server_create, freed by farpca_server_destroy: the only device
 * allocation the library makes), `slots` streams, a scheduler thread and one
 * finisher thread per stream.  farpca_server_submit queues a request whose A is already
 * resident (caller-owned, read only, valid until the request's result is
 * polled).  The scheduler keeps up to `slots` solves in flight, each on its own
 * stream, and advances them one block at a time (farpca_step_async /
 * farpca_step_poll), so that the blocks of all admitted solves interleave on the
 * device.  Memory is granted by blocks: a request is admitted once the loop part
 * for its first four blocks fits (farpca_loop_bytes), its loop part is moved to
 * one twice as large whenever its next block needs room (farpca_grow), and the
 * final part plus the outputs U, S, V, sized for the columns the solve returns,
 * are granted when its block loop ends (a finisher thread runs the final step).
 * The queue is scanned in arrival order and the first request that fits is
 * admitted, unless an earlier one has waited more than starve_s seconds (then
 * nothing overtakes it).  If every solve in flight waits for memory and nothing
 * else can free any, the solve admitted last goes back to the head of the queue
 * and runs again later from its first block.  A result (U, S, V inside the pool,
 * leading dimension ld = rank_out) stays valid until farpca_server_release(tag).
 * Results are bitwise the same whether a request runs alone, among others, or
 * through farpca_run.  Tags must be unique among queued, running and unreleased
 * requests.  Times are seconds since the server was created (steady clock).
 * The kernel-timing switch below must be off while a server runs. */
typedef struct farpca_result {
  uint64_t tag;
  int32_t status;        /* the solve's status (as farpca_run would return it)          */
  int32_t reserved0;
  farpca_info info;
  double t_submit, t_admit, t_done;
  float *dU;             /* m x info.rank_out of an m x ld array (device, in the pool)  */
  double *dS;            /* info.rank_out singular values, descending                  */
  float *dV;             /* n x info.rank_out of an n x ld array                       */
  int64_t ld, m, n;
} farpca_result;
typedef struct farpca_server_s farpca_server_t;
size_t farpca_request_footprint(const farpca_params *params);   /* 0 if the params are invalid */
int farpca_server_create(size_t pool_bytes, int slots, double starve_s, farpca_server_t **out);
/* farpca_request_footprint: the most a request can hold (every block, the final part for
 * l_max, U S V for l_max columns).  Submit returns FARPCA_E_NOMEM when that can never fit
 * the pool, FARPCA_E_INVALID for bad params or tag. */
int farpca_server_submit(farpca_server_t *srv, const farpca_params *params, const void *dA,
                         uint64_t tag);
/* Up to max_out finished results (waits up to wait_ms for the first); returns the count. */
int farpca_server_poll(farpca_server_t *srv, farpca_result *out, int max_out, int wait_ms);
int farpca_server_release(farpca_server_t *srv, uint64_t tag);
/* Copy a held result's first info.rank_out columns into caller buffers (device,
 * row-major, ldu / ldv >= rank_out; any of the three may be NULL), enqueued on `stream`. */
int farpca_server_fetch(farpca_server_t *srv, const farpca_result *res, float *dU, int64_t ldu,
                        double *dS, float *dV, int64_t ldv, void *stream);
int farpca_server_stats(farpca_server_t *srv, int *queued, int *running, size_t *largest_free);
/* Pool bytes granted now and at most so far, loop parts moved to larger ones,
 * solves put back in the queue for want of memory (any pointer may be NULL). */
int farpca_server_memory(farpca_server_t *srv, size_t *in_use, size_t *peak, int64_t *grows,
                         int64_t *preemptions);
/* Waits for running requests, drops queued ones, frees the pool (results become invalid). */
int farpca_server_destroy(farpca_server_t *srv);

/* ---- opt-in kernel timing (process-wide, not thread-safe): while enabled,
 * farpca_run records hipEvents on its stream around the kernels that stream A
 * and, on return, adds their elapsed times per class.  Enabling resets the
 * totals.  Events cost a few microseconds per launch; leave off in production. */
#define FARPCA_PROF_SKETCH 0   /* sparse sketch kernel (partials not included)   */
#define FARPCA_PROF_GEMM_TN 1  /* A^T T products of the power steps              */
#define FARPCA_PROF_GEMM_NN 2  /* A G products (and the Gaussian sketch)        */
#define FARPCA_PROF_EIG 3      /* final FP64 eigendecomposition                 */
#define FARPCA_PROF_GEMM_C 4   /* C_j^T = A^T Q_j (kept in C^T, summed in E)    */
#define FARPCA_PROF_NCLASS 5
void farpca_profile_enable(int on);
int farpca_profile_get(int cls, double *total_ms, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* FARPCA_H_ */
