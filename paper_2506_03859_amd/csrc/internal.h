// Internal launch interfaces shared by the HIP translation units and the
// host orchestration.  Not part of the public C-ABI (include/farpca.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

struct farpca_plan_s;   // the plan (farpca.cpp)

namespace farpca_int {

constexpr int kMaxBlock = 64;   // block size b <= 64 (one 64-bit mask per row of Omega)
constexpr int kChunk = 64;      // rows of Omega (columns of A) per sketch chunk
constexpr int kBld = 64;        // leading dimension of every n x b / m x b block buffer

enum SketchKind { SK_GAUSSIAN = 0, SK_STD_BERNOULLI = 1, SK_SPARSE_SIGN = 2,
                  SK_SPARSE_GAUSSIAN = 3, SK_BERNOULLI = 4 };

struct OmegaSpec {
  int kind;            // SketchKind
  int b;               // block size
  int zeta;            // fixed-count sparse sign (0: i.i.d.)
  uint32_t thr;        // floor(p * 2^32) for the i.i.d. kinds
  double dense_scale;  // value scale in the dense copy (1/sqrt(zeta), 1/sqrt(p), ...)
  double p;            // Bernoulli parameter (standardized Bernoulli: dense copy holds B - p)
  uint64_t seed;
};

// One entry of a chunk's column list: byte offset of the Omega row inside the
// staged A tile, and the unscaled value (+-1, 1 or a Gaussian draw).  Every
// column's list is padded with zero-valued entries to a multiple of
// kListPad, so the sketch consumes whole groups; kEntCap entries per chunk.
// The lists use at most kChunk * kMaxBlock + (kListPad - 1) * kMaxBlock
// slots; the 128 + kMaxBlock slots after them are room for the sketch's
// fixed-size reads past a list's end (never used as entries).
struct ChunkEntry { uint32_t lds_off; float val; };
constexpr int kListPad = 4;
constexpr int kEntCap = kChunk * kMaxBlock + kListPad * kMaxBlock + 128;

// ---- omega.hip
// Generates Omega_j for rows [0, n): mask/sign words (n each), the dense copy
// (n x kBld, columns >= b zero) and, if `entries` is non-null, the per-chunk
// column lists: colptr[(chunk)*(kMaxBlock+1) + c], entries[chunk*kEntCap + e].
void launch_omega(const OmegaSpec &s, int64_t n, int64_t block_j,
                  uint64_t *mask_out, uint64_t *sign_out, float *dense_out,
                  uint32_t *colptr, ChunkEntry *entries, int lds_row_stride_bytes,
                  hipStream_t st);

// ---- sketch.hip
// nsplit == 1: out (m x kBld) = scale * (A Omega) + zc * z (z may be null).
// nsplit > 1: out = partials (nsplit x m x kBld) of the unscaled sums over
// consecutive chunk groups; finish with launch_reduce_partials.
// A is FP32 or (bf16) BF16 bit patterns.
void launch_sketch_full(const void *A, bool bf16, int64_t lda, int64_t m, int64_t n, int b,
                        const uint32_t *colptr, const ChunkEntry *entries, float *out,
                        int nsplit, float scale, const float *z, float zc, hipStream_t st);
int sketch_choose_split(int64_t m, int64_t n);
int sketch_lds_row_stride_bytes();
int sketch_rows_per_wg();

// ---- sketch_cols.hip (A stored column-major: element (i, k) at A[k * lda + i])
// One list per column c < b of Omega_j from the per-chunk lists of
// launch_omega (generated with row stride 1): flat[c * n + e] = (row of
// Omega_j, value), ascending row, colcnt[c] entries.
void launch_flatten_lists(const uint32_t *colptr, const ChunkEntry *entries, int64_t n, int b,
                          ChunkEntry *flat, uint32_t *colcnt, hipStream_t st);
// out (m x kBld) = scale * (A Omega_j) + zc * z (z may be null); columns >= b zero.
void launch_sketch_cols(const float *A, int64_t lda, int64_t m, int64_t n, int b,
                        const ChunkEntry *flat, const uint32_t *colcnt, float *out, float scale,
                        const float *z, float zc, hipStream_t st);
// rowsum[i] = sum_k A[i][k] (FP64) for column-major A (m x n); `part` holds
// colsum_num_splits(m, n) x m doubles.
int colsum_num_splits(int64_t m, int64_t n);
void launch_colsum(const float *A, int64_t lda, int64_t m, int64_t n, double *part, double *rowsum,
                   hipStream_t st);

// ---- gemm.hip (FP32 MFMA, FP32 accumulation)
// NN: C[M x N] = A[M x K] * X[K x N]; A row-major (lda), X row-major (ldx).
// TN: C[M x N] = A^T * Y with A K x M row-major (lda), Y K x N row-major (ldy).
// N <= 64 per call.  With ksplit > 1 the kernel writes ksplit partial
// products to `part` (ksplit x M x ldc_part) and reduce_partials finishes.
// Without split it writes C directly: C = alpha*AB + beta*C.
void launch_gemm_nn(const float *A, int64_t lda, const float *X, int64_t ldx,
                    float *C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                    float alpha, float beta, int ksplit, float *part, hipStream_t st);
void launch_gemm_tn(const float *A, int64_t lda, const float *Y, int64_t ldy,
                    float *C, int64_t ldc, int64_t M, int64_t N, int64_t K,
                    float alpha, float beta, int ksplit, float *part, hipStream_t st);
// C[i][c] = alpha * sum_s part[s][i][c] + beta * C[i][c] + gamma * D[i][c] + zc * z[i]
// (D, z optional; fixed summation order).
void launch_reduce_partials(const float *part, int nsplit, int64_t M, int64_t N,
                            float *C, int64_t ldc, float alpha, float beta,
                            const float *D, int64_t ldd, float gamma,
                            const float *z, float zc, hipStream_t st);
// K splits for an M-row product over K; the partial buffer holds at least
// max_split x M x kBld floats.
int gemm_choose_ksplit(int64_t M, int64_t K, int is_tn, int64_t max_split);
// The same products split in two launches: the main kernel (returns the number
// of K splits it wrote) and the fixed-order reduction of the partials.
int launch_gemm_nn_main(const float *A, int64_t lda, const float *X, int64_t ldx, float *C,
                        int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                        int ksplit, float *part, hipStream_t st);
int launch_gemm_tn_main(const float *A, int64_t lda, const float *Y, int64_t ldy, float *C,
                        int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                        int ksplit, float *part, hipStream_t st);
void launch_gemm_finish(const float *part, int nsp, int64_t M, int64_t N, float *C, int64_t ldc,
                        float alpha, float beta, hipStream_t st);

// ---- gemm_bf16.hip (A stored as BF16 bit patterns; the FP32 skinny operand
// is split exactly into three BF16 terms; FP32 accumulation).  Same NN / TN
// conventions and partial handling as the FP32 kernels.  `xt` is scratch of
// bf16_pack_bytes(K) bytes (the transposed, zero-padded skinny operand).
int64_t bf16_padded_k(int64_t K);
size_t bf16_pack_bytes(int64_t K);
int gemm_bf16_choose_ksplit(int64_t M, int64_t K, int is_tn, int64_t max_split);
int launch_gemm_bf16_nn_main(const uint16_t *A, int64_t lda, const float *X, int64_t ldx, float *C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                             int ksplit, float *part, float *xt, hipStream_t st);
int launch_gemm_bf16_tn_main(const uint16_t *A, int64_t lda, const float *Y, int64_t ldy, float *C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                             int ksplit, float *part, float *xt, hipStream_t st);
// The same products with FP32 A on the BF16 matrix cores: A is split exactly
// into three BF16 terms in registers as well, and six of the nine term
// products are formed (the three left out are below 2^-23 of |a x| and of
// either sign).
int gemm_f32s_choose_ksplit(int64_t M, int64_t K, int is_tn, int64_t max_split);
int launch_gemm_f32s_nn_main(const float *A, int64_t lda, const float *X, int64_t ldx, float *C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                             int ksplit, float *part, float *xt, hipStream_t st);
int launch_gemm_f32s_tn_main(const float *A, int64_t lda, const float *Y, int64_t ldy, float *C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                             int ksplit, float *part, float *xt, hipStream_t st);

// ---- dense64.hip (FP64 small-matrix work)
// Gram G[b x b] (FP64) = X^T X for X (K x b, FP32, ldx; columns >= b ignored);
// partials in `part` (nblk x 64 x 64 doubles), nblk = gram_num_partials(K) <=
// gram_max_partials().
int gram_num_partials(int64_t K);
int gram_max_partials();
void launch_gram(const float *X, int64_t ldx, int64_t K, int b, double *part, double *G,
                 hipStream_t st);
// Cholesky factor G = R^T R (64 x 64 FP64): F = R strictly above the
// diagonal, 1 / R_jj on it.  Columns whose pivot is <= drop_rel * diagonal
// are dropped (zero row of R, F_jj = 0); flags[0] |= 1 then.  skip_tol > 0
// (a repeated pass): if every kept column of G is orthonormal to skip_tol,
// nothing is factored and apply[0] = 0, else apply[0] = 1 (apply may be null
// when skip_tol == 0).
void launch_chol(const double *G, int b, double drop_rel, double *F, int *flags, double skip_tol,
                 int *apply, hipStream_t st);
// Y = X R^{-1} row by row (forward substitution in FP64; in place allowed);
// nothing is done when apply is non-null and apply[0] == 0 (requires Y == X).
void launch_trsm_rows(const float *X, int64_t ldx, int64_t K, int b, const double *F, float *Y,
                      int64_t ldy, const int *apply, hipStream_t st);
// Setup pass over A: partial sums of squares (FP64, per row block) and the
// row sums (FP64, rowsum[i]); nonfinite flag.
int setup_num_partials(int64_t m);
void launch_setup(const void *A, bool bf16, int64_t lda, int64_t m, int64_t n, double *part_sq,
                  double *rowsum, int *flags, hipStream_t st);
// out[0] = sum of partials (fixed order).
void launch_sum_partials(const double *part, int count, double *out, hipStream_t st);
// z[i] = (float)(p * rowsum[i])
void launch_scale_rowsum(const double *rowsum, int64_t m, double p, float *z, hipStream_t st);
// ||X||_F^2 of X (K x b, FP32) into partials (one double per block) for the indicator.
int sqnorm_num_partials(int64_t K);
void launch_sqnorm(const float *X, int64_t ldx, int64_t K, int b, double *part, hipStream_t st);

// ---- cpass64.hip
// C (M x b, FP32, ldc) = A^T Q (row-major A: m x n, M = n, K = m; colmajor:
// A stored as A^T row-major) with FP64 products and sums; part holds
// nsplit x M x kBld doubles; sq gets sqnorm_num_partials(M) FP64 partials of
// ||C||_F^2 taken before the rounding to FP32.
int cpass64_choose_split(int64_t M, int64_t K, int64_t max_split);
void launch_cpass64(const void *A, bool bf16, bool colmajor, int64_t lda, const float *Q, int64_t ldq,
                    int64_t M, int64_t K, int b, int nsplit, double *part, float *C, int64_t ldc,
                    double *sq, hipStream_t st);
// E_hist[j] = E_prev - sum(part); E_cur updated (single thread).
void launch_indicator_update(const double *part, int count, double *E, double *E_hist,
                             int64_t j, hipStream_t st);
// Copy a K x b FP32 block (ld ldx) into dst (ld ldd).
void launch_copy_block(const float *X, int64_t ldx, int64_t K, int b, float *dst, int64_t ldd,
                       hipStream_t st);
// X -= alpha * G (K x b)
void launch_axpy_block(float *X, int64_t ldx, const float *G, int64_t ldg, int64_t K, int b,
                       const double *alpha_dev, hipStream_t st);
// Shift update from the descending eigenvalues w of the block Gram.
void launch_alpha_update(const double *w, int b, double *alpha, hipStream_t st);

// ---- eig.hip (FP64 symmetric eigensolver, block Jacobi)
size_t eig_workspace_bytes(int64_t l);
// Eigen-decomposition of the symmetric l x l matrix K (FP64, row-major, ld l):
// eigenvalues descending in w[l], eigenvectors in Vout (l x l row-major, column
// i <-> w[i]).  Returns number of sweeps used (host-synchronous).
// Off-diagonal entries are reduced until |a_pq| <= rel sqrt(|a_pp a_qq|) (or
// an absolute floor); rel <= 0 selects the default 1e-14.  *converged (if
// given) is false when the test still failed after kEigMaxSweeps sweeps.
constexpr int kEigMaxSweeps = 40;
int eig_sym(const double *K, int64_t l, double *w, double *Vout, void *work, double rel,
            hipStream_t st, bool *converged = nullptr);
// Single-workgroup Jacobi for s <= 64 (used for the b x b Gram in the shift).
// conv (device, may be null): 1 if the sweeps converged, 0 if they hit the cap.
void launch_eig_small(const double *K, int s, int ldk, double *w, double *Vout, int ldv,
                      hipStream_t st, int *conv = nullptr);
// Y[r][c] = (float)(X[r][c] * f(c)), f(c) = 1 (s null) or 1/s[c] (0 if s[c] == 0).
void launch_convert_f64_f32(const double *X, int64_t rows, int64_t cols, int64_t ldx,
                            const double *s, float *Y, int64_t ldy, hipStream_t st);
void launch_sqrt_clip(const double *w, int64_t l, double *s, hipStream_t st);
// rank_trunc of farpca_info into out[0] (device): see trunc_rank_kernel.
void launch_trunc_rank(const double *s, int64_t k, const double *scal, double tol, bool fixed,
                       int64_t *out, hipStream_t st);

// ---- gram64 (big FP64 Gram for the final step): K = X^T X, X n x l FP32 (ldx)
size_t gram_big_workspace_bytes(int64_t n, int64_t l);
// `work_bytes` bounds the partial buffers (the split count is reduced to fit).
void launch_gram_big(const float *X, int64_t ldx, int64_t n, int64_t l, double *K,
                     void *work, size_t work_bytes, hipStream_t st);

// ---- farpca.cpp (plan accessors for the server)
// blocks a run may reach (l_max / b)
int64_t plan_max_blocks(const ::farpca_plan_s *plan);
// columns the final step writes (the fixed rank k, else the reached l; 0 before any block)
int64_t plan_rank_out(const ::farpca_plan_s *plan);

}  // namespace farpca_int
