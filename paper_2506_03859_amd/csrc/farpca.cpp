// Host orchestration and C-ABI of the accelerated farPCA loop (Algorithm 1 /
// Algorithm 2 of arXiv 2506.03859) on one gfx950 GPU.
//
// Per block j (b columns):
//   Omega_j from the counter-based generator (Definitions 2.1-2.4)
//   S   = A Omega_j                 sparse gather kernel (dense MFMA product for
//                                   the Gaussian matrix); standardized Bernoulli:
//                                   A B_j - z, z = A (p 1_n) (Section 3.1)
//   P >= 1, k = 1..P:
//     T  <- (I - Q Q^T) T  (twice)   T = S for k = 1, T = A G otherwise
//     X   = A^T T - alpha G          = A^T(AG) - W Z^{-1} W^T G - alpha G of
//                                   Algorithm 1, evaluated with the orthonormal
//                                   basis Q of Y (W Z^{-1} W^T = A^T Q Q^T A)
//     G   = orth(X)                  CholeskyQR (2 passes, FP64 Gram); the shift
//                                   update uses the block's smallest singular
//                                   value (P > 2)
//   Y_j = A G (P >= 1) or S (P = 0)
//   Y_j <- (I - Q Q^T) Y_j (twice), one CholeskyQR pass, (I - Q Q^T) once
//   more, a second pass: Q_j = orth(Y_j), Q = [Q, Q_j]
//   C_j^T = A^T Q_j, E = E - ||C_j||_F^2   (E = ||A||^2 - tr(T Z^{-1}) of
//                                   Algorithm 1, since tr(T Z^{-1}) = ||Q^T A||_F^2)
//   stop when E < tol^2 ||A||_F^2 (Section 5.2), l >= k (Section 5.1) or at the cap.
// Final: K = C C^T (FP64), K = U~ diag(lambda) U~^T (Jacobi), Sigma = lambda^{1/2},
//        U = Q U~, V = C^T U~ Sigma^{-1}  (the final steps of Algorithm 1 up to a
//        rotation of the basis).
// Every step runs in a kernel of this library; the host only sequences
// launches and reads E (8 bytes) after each block.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "../../include/farpca.h"
#include "internal.h"

using namespace farpca_int;

// squared relative pivot below which a block direction counts as dependent
static constexpr double kDropRel = 1e-10;
// Below this tolerance the stop test (E < tol^2 ||A||^2) is within about two
// orders of magnitude of the error that FP32 accumulation leaves in
// sum ||C_j||^2 (1e-8 .. 1e-7 of ||A||^2), and C_j^T = A^T Q_j is formed with
// FP64 products and sums instead.
static constexpr double kC64Tol = 1e-3;
static constexpr int kCholqrPasses = 2;
// a repeated CholeskyQR pass is skipped when the Gram of its input deviates
// from the identity by at most this much (orthonormal far beyond what the
// FP32 data and the method need)
static constexpr double kRepeatSkip = 1e-8;
// Final eigensolve of K = C C^T: Jacobi stops once every off-diagonal entry is
// below 1e-7 of the geometric mean of its two diagonal entries.  The
// eigenvalues are then exact to FP64 rounding (their error is quadratic in the
// off-diagonal entries); V = C^T U~ Sigma^{-1} is orthonormal to the same 1e-7,
// about the rounding of its FP32 entries, and U S V^T = Q Q^T A holds for any
// orthogonal U~, so FP32 outputs lose nothing.
static constexpr double kFinalEigRel = 1e-7;

struct farpca_plan_s {
  farpca_params prm;
  bool bf16;            // A holds BF16 bit patterns (precision form)
  bool colmajor;        // A stored column-major (FARPCA_LAYOUT_COL)
  bool c64;             // C_j^T = A^T Q_j with FP64 accumulation (tol below kC64Tol)
  bool split;           // A-passes on the BF16 matrix cores with both operands split (FP32 row-major A)
  int b;
  int P;
  int kind;
  int zeta;
  double p;
  uint32_t thr;
  double dense_scale;   // scale of Omega's nonzeros in the dense copy
  float sketch_scale;   // scale applied to the sketch sums
  int64_t maxblk;
  int64_t lmax;
  int64_t nchunks;
  // Workspace layout (byte offsets).  The loop part holds what the block
  // loop needs, with Q and C^T sized for `cap` blocks (leading dimension ldq);
  // the final part (step a10) is sized for the basis the run reached.  A full
  // workspace (farpca_run) is the loop part for every block, then the final
  // part for l_max at off_final.
  int64_t cap;          // blocks Q and C^T have room for in the loop layout
  int64_t ldq;          // leading dimension of Q and C^T (cap b rounded to 4)
  size_t off_q, off_ct, off_s, off_y, off_x, off_g, off_om, off_mask, off_neg, off_colptr,
      off_ent, off_z, off_rowsum, off_r, off_part, off_gpart, off_g64, off_rinv, off_w64,
      off_v64, off_setup, off_sq, off_scal, off_ehist, off_xt, off_flat, off_colcnt, loop_bytes;
  size_t off_final, total;
  int64_t part_floats;  // capacity of the K-split partial buffer
  // state of a run between farpca_begin and farpca_finish (host side)
  int stage = 0;        // 0 idle, 1 blocks running, 2 block loop done
  const void *run_a = nullptr;
  char *run_work = nullptr;     // loop part of the running solve
  char *run_final = nullptr;    // final part inside a full workspace (null: given at finish)
  size_t run_work_bytes = 0;
  bool own_ehist = true;        // the E history lives in the loop part
  double *run_ehist = nullptr;
  double norm_a2 = 0.0, stop_thr = 0.0;   // ||A||_F^2, tol^2 ||A||_F^2
  int64_t l = 0;
  int blocks = 0;
  int status = FARPCA_NOT_CONVERGED;
  // a block enqueued by farpca_step_async whose E read-back has not been
  // examined yet; the read-back lands in pinned host memory, its completion is
  // marked by an event (both created on first use, released by farpca_free)
  bool step_pending = false;
  double *h_e = nullptr;
  hipEvent_t ev_step = nullptr;
  // K splits the partial buffer holds for an M-row product
  int64_t part_splits(int64_t M) const { return M > 0 ? part_floats / (M * kBld) : 1; }
};

namespace {

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

struct Carver {
  size_t cur = 0;
  size_t take(size_t bytes) {
    const size_t o = cur;
    cur = align_up(cur + bytes);
    return o;
  }
};

#define HIP_OK(x)                                   \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) return FARPCA_E_DEVICE;   \
  } while (0)

int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }

struct Ws {
  char *base;
  template <typename T>
  T *at(size_t off) const { return reinterpret_cast<T *>(base + off); }
};

// Final part (step a10) for an l-column basis: K = C C^T, the eigensolver's
// scratch, eigenvalues, eigenvectors (FP64 and FP32), the Gram partials.
struct FinalLayout {
  size_t kbig, eig, wfin, vfin, u32, gbig, gbig_bytes, total;
};
FinalLayout final_layout(int64_t n, int64_t l) {
  FinalLayout f;
  Carver c;
  f.kbig = c.take((size_t)l * l * 8);
  f.eig = c.take(eig_workspace_bytes(l));
  f.wfin = c.take((size_t)l * 8);
  f.vfin = c.take((size_t)l * l * 8);
  f.u32 = c.take((size_t)l * l * 4);
  f.gbig_bytes = gram_big_workspace_bytes(n, l);
  f.gbig = c.take(f.gbig_bytes);
  f.total = c.cur;
  return f;
}

}  // namespace

// Loop part for a capacity of cap blocks: sets ldq and the loop offsets,
// returns its size.
static size_t carve_loop(farpca_plan_s *pl, int64_t cap) {
  const farpca_params &q = pl->prm;
  const int64_t m = q.m, n = q.n, b = pl->b;
  pl->cap = cap;
  pl->ldq = (cap * b + 3) / 4 * 4;
  const int64_t ldq = pl->ldq;
  const int64_t mnl = imax(imax(m, n), pl->lmax);
  Carver c;
  pl->off_q = c.take((size_t)m * ldq * 4);
  pl->off_ct = c.take((size_t)n * ldq * 4);
  pl->off_s = c.take((size_t)m * kBld * 4);
  pl->off_y = c.take((size_t)m * kBld * 4);
  pl->off_x = c.take((size_t)n * kBld * 4);
  pl->off_g = c.take((size_t)n * kBld * 4);
  pl->off_om = c.take((size_t)n * kBld * 4);
  pl->off_mask = c.take((size_t)n * 8);
  pl->off_neg = c.take((size_t)n * 8);
  pl->off_colptr = c.take((size_t)pl->nchunks * (kMaxBlock + 1) * 4);
  pl->off_ent = c.take((size_t)pl->nchunks * kEntCap * sizeof(ChunkEntry));
  pl->off_z = c.take((size_t)m * 4);
  pl->off_rowsum = c.take((size_t)imax(m, n) * 8);   // column-major setup: n stored rows
  pl->off_r = c.take((size_t)ldq * kBld * 4);
  pl->part_floats = 16 * mnl * kBld;
  pl->off_part = c.take((size_t)pl->part_floats * 4);
  pl->off_gpart = c.take((size_t)gram_max_partials() * kMaxBlock * kMaxBlock * 8);
  pl->off_g64 = c.take((size_t)kMaxBlock * kMaxBlock * 8);
  pl->off_rinv = c.take((size_t)kMaxBlock * kMaxBlock * 8);
  pl->off_w64 = c.take((size_t)kMaxBlock * 8);
  pl->off_v64 = c.take((size_t)kMaxBlock * kMaxBlock * 8);
  pl->off_setup = c.take((size_t)imax(setup_num_partials(m), setup_num_partials(n)) * 8);
  pl->off_sq = c.take((size_t)256 * 8);                               // <= 256 partials for any K
  pl->off_scal = c.take(64);                        // nA2, E, alpha, flags, truncation rank
  pl->off_ehist = c.take((size_t)pl->maxblk * 8);
  pl->off_xt = (pl->bf16 || pl->split) ? c.take(bf16_pack_bytes(imax(m, n))) : 0;
  // column-major: one list per column of Omega_j over all n rows
  pl->off_flat = pl->colmajor ? c.take((size_t)b * n * sizeof(ChunkEntry)) : 0;
  pl->off_colcnt = pl->colmajor ? c.take((size_t)kMaxBlock * 4) : 0;
  pl->loop_bytes = c.cur;
  return c.cur;
}

// The layout of a full workspace (every block, final part for l_max).
static void carve_full(farpca_plan_s *pl) {
  pl->off_final = carve_loop(pl, pl->maxblk);
  pl->total = pl->off_final + final_layout(pl->prm.n, pl->lmax).total;
}

extern "C" const char *farpca_status_str(int status) {
  switch (status) {
    case FARPCA_OK: return "ok";
    case FARPCA_NOT_CONVERGED: return "block cap reached before the tolerance";
    case FARPCA_E_INVALID: return "invalid parameter";
    case FARPCA_E_NOMEM: return "workspace too small";
    case FARPCA_E_DEVICE: return "HIP error";
    case FARPCA_E_NONFINITE: return "A holds NaN or Inf";
    default: return "unknown status";
  }
}

extern "C" int farpca_plan(const farpca_params *prm, farpca_plan_t **out, int64_t *l_max,
                           size_t *workspace_bytes) {
  if (!prm || !out) return FARPCA_E_INVALID;
  *out = nullptr;
  const farpca_params &q = *prm;
  if (q.a_layout != FARPCA_LAYOUT_ROW && q.a_layout != FARPCA_LAYOUT_COL) return FARPCA_E_INVALID;
  const bool colmajor = q.a_layout == FARPCA_LAYOUT_COL;
  if (q.m < 1 || q.n < 1 || q.lda < (colmajor ? q.m : q.n)) return FARPCA_E_INVALID;
  if (q.a_dtype != FARPCA_DTYPE_F32 && q.a_dtype != FARPCA_DTYPE_BF16) return FARPCA_E_INVALID;
  if (colmajor && q.a_dtype != FARPCA_DTYPE_F32) return FARPCA_E_INVALID;
  if (q.sketch < FARPCA_GAUSSIAN || q.sketch > FARPCA_BERNOULLI) return FARPCA_E_INVALID;
  if (q.block < 0 || q.block > kMaxBlock || q.power < 0 || q.power > 64) return FARPCA_E_INVALID;
  if (q.rank < 0 || q.max_blocks < 0) return FARPCA_E_INVALID;
  if (q.rank == 0 && !(q.tol > 0.0 && std::isfinite(q.tol))) return FARPCA_E_INVALID;
  if (!(q.sketch_p >= 0.0 && q.sketch_p < 1.0)) return FARPCA_E_INVALID;
  const int64_t mn = imin(q.m, q.n);
  int b = q.block ? q.block : (int)imin(imax(20, mn / 100), 50);
  if (b > mn) {
    if (q.block) return FARPCA_E_INVALID;
    b = (int)mn;
  }
  if (q.sketch_zeta < 0 || q.sketch_zeta > b) return FARPCA_E_INVALID;

  farpca_plan_s *pl = new (std::nothrow) farpca_plan_s();
  if (!pl) return FARPCA_E_INVALID;
  pl->prm = q;
  pl->bf16 = q.a_dtype == FARPCA_DTYPE_BF16;
  pl->colmajor = colmajor;
  pl->c64 = q.tol > 0.0 && q.tol < kC64Tol;
  pl->split = !pl->bf16 && !colmajor;
  pl->b = b;
  pl->P = q.power;
  pl->kind = q.sketch;
  pl->zeta = (q.sketch == FARPCA_SPARSE_SIGN) ? q.sketch_zeta : 0;
  double p = q.sketch_p;
  if (p == 0.0) {
    // Section 5's rules with N the number of rows of Omega_j (the columns of A):
    // about ln N (p1) or 10 (p2) nonzeros per column of the test matrix
    const double N = (double)q.n;
    p = (q.sketch == FARPCA_STD_BERNOULLI) ? std::fmax(1e-3, std::log(N) / N)
                                           : std::fmax(1e-3, 10.0 / N);
  }
  pl->p = p;
  const double tp = std::floor(p * 4294967296.0);
  const bool uses_p = q.sketch != FARPCA_GAUSSIAN && pl->zeta == 0;
  if (uses_p && tp < 1.0) { delete pl; return FARPCA_E_INVALID; }
  pl->thr = (uint32_t)(tp >= 4294967295.0 ? 4294967295.0 : tp);
  switch (q.sketch) {
    case FARPCA_SPARSE_SIGN:
      pl->dense_scale = pl->zeta ? 1.0 / std::sqrt((double)pl->zeta) : 1.0 / std::sqrt(p);
      break;
    case FARPCA_SPARSE_GAUSSIAN: pl->dense_scale = 1.0 / std::sqrt(p); break;
    default: pl->dense_scale = 1.0; break;
  }
  pl->sketch_scale = (float)pl->dense_scale;

  int64_t maxblk = q.max_blocks ? q.max_blocks : (mn + 2 * b - 1) / (2 * b);
  if (q.rank > 0) maxblk = (q.rank + b - 1) / b;
  maxblk = imin(maxblk, mn / b);
  if (maxblk < 1) maxblk = 1;
  pl->maxblk = maxblk;
  pl->lmax = maxblk * b;
  pl->nchunks = (q.n + kChunk - 1) / kChunk;
  carve_full(pl);
  if (colmajor && (int64_t)colsum_num_splits(q.m, q.n) * q.m * 2 > pl->part_floats) {
    delete pl;
    return FARPCA_E_INVALID;
  }
  *out = pl;
  if (l_max) *l_max = pl->lmax;
  if (workspace_bytes) *workspace_bytes = pl->total;
  return FARPCA_OK;
}

namespace farpca_int {
int64_t plan_max_blocks(const ::farpca_plan_s *plan) { return plan ? plan->maxblk : 0; }
int64_t plan_rank_out(const ::farpca_plan_s *plan) {
  if (!plan || plan->blocks == 0) return 0;
  return plan->prm.rank > 0 ? imin(plan->prm.rank, plan->l) : plan->l;
}
}  // namespace farpca_int

extern "C" void farpca_free(farpca_plan_t *plan) {
  if (!plan) return;
  if (plan->ev_step) {
    hipEventSynchronize(plan->ev_step);
    hipEventDestroy(plan->ev_step);
  }
  if (plan->h_e) hipHostFree(plan->h_e);
  delete plan;
}

namespace {

// Opt-in event timing of the kernels that stream A (hipEvents recorded on the
// caller's stream around each launch; resolved when farpca_run returns).
struct ProfClass { double total_ms = 0.0; int64_t count = 0; };
struct Prof {
  bool on = false;
  ProfClass cls[FARPCA_PROF_NCLASS];
  struct Pending { hipEvent_t a, b; int c; };
  Pending pend[4096];
  int npend = 0;
};
Prof g_prof;

struct ProfScope {
  hipStream_t st;
  int c;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(int cls, hipStream_t s) : st(s), c(cls) {
    if (!g_prof.on || g_prof.npend >= 4096) return;
    if (hipEventCreate(&a) != hipSuccess) { a = nullptr; return; }
    if (hipEventCreate(&b) != hipSuccess) { hipEventDestroy(a); a = nullptr; return; }
    hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a) return;
    hipEventRecord(b, st);
    g_prof.pend[g_prof.npend++] = {a, b, c};
  }
};

void prof_resolve() {
  for (int i = 0; i < g_prof.npend; ++i) {
    auto &p = g_prof.pend[i];
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      g_prof.cls[p.c].total_ms += ms;
      g_prof.cls[p.c].count += 1;
    }
    hipEventDestroy(p.a);
    hipEventDestroy(p.b);
  }
  g_prof.npend = 0;
}

OmegaSpec omega_spec(const farpca_plan_s *pl) {
  OmegaSpec s;
  s.kind = pl->kind;
  s.b = pl->b;
  s.zeta = pl->zeta;
  s.thr = pl->thr;
  s.dense_scale = pl->dense_scale;
  s.p = pl->p;
  s.seed = pl->prm.seed;
  return s;
}

// Omega_j into the workspace (dense copy, masks, column lists).
void gen_omega(const farpca_plan_s *pl, const Ws &w, int64_t j, hipStream_t st,
               uint64_t *mask = nullptr, uint64_t *neg = nullptr, float *dense = nullptr) {
  const bool lists = pl->kind != FARPCA_GAUSSIAN;
  // row-major: entry offsets address the sketch's LDS tile; column-major:
  // rows inside the chunk, flattened into one list per column
  launch_omega(omega_spec(pl), pl->prm.n, j, mask ? mask : w.at<uint64_t>(pl->off_mask),
               neg ? neg : w.at<uint64_t>(pl->off_neg),
               dense ? dense : (lists ? nullptr : w.at<float>(pl->off_om)),   // dense copy: Gaussian product only
               lists ? w.at<uint32_t>(pl->off_colptr) : nullptr,
               lists ? w.at<ChunkEntry>(pl->off_ent) : nullptr,
               pl->colmajor ? 1 : sketch_lds_row_stride_bytes(), st);
  if (lists && pl->colmajor)
    launch_flatten_lists(w.at<uint32_t>(pl->off_colptr), w.at<ChunkEntry>(pl->off_ent), pl->prm.n,
                         pl->b, w.at<ChunkEntry>(pl->off_flat), w.at<uint32_t>(pl->off_colcnt), st);
}

// Setup pass over A (step a0): partial sums of squares, finiteness flag and,
// for the standardized Bernoulli matrix, the row sums of A.  Column-major A is
// passed to the row-major setup as the n x m stored matrix (same squares and
// flag); its row sums come from a column-sum pass.
void setup_pass(const farpca_plan_s *pl, const Ws &w, const void *A, int *flags, hipStream_t st) {
  const farpca_params &q = pl->prm;
  double *rowsum = w.at<double>(pl->off_rowsum);
  if (!pl->colmajor) {
    launch_setup(A, pl->bf16, q.lda, q.m, q.n, w.at<double>(pl->off_setup), rowsum, flags, st);
    return;
  }
  launch_setup(A, false, q.lda, q.n, q.m, w.at<double>(pl->off_setup), rowsum, flags, st);
  if (pl->kind == FARPCA_STD_BERNOULLI)
    launch_colsum(static_cast<const float *>(A), q.lda, q.m, q.n,
                  reinterpret_cast<double *>(w.at<float>(pl->off_part)), rowsum, st);
}

int setup_partials(const farpca_plan_s *pl) {
  return setup_num_partials(pl->colmajor ? pl->prm.n : pl->prm.m);
}

// One A-pass with the plan's storage type of A, split over K:
//   NN (tn false): C (m x ncols) = A X, X n x ncols (ld kBld)
//   TN (tn true):  C (n x ncols) = A^T T, T m x ncols (ld kBld)
// Returns the number of partial products left in the partial buffer (1: C
// was written directly); launch_gemm_finish completes the product.  With FP32
// row-major A the pass runs split on the BF16 matrix cores.
int a_pass(const farpca_plan_s *pl, const Ws &w, bool tn, const void *A, const float *X, int ncols,
           float *C, int64_t ldc, hipStream_t st) {
  const farpca_params &q = pl->prm;
  float *part = w.at<float>(pl->off_part);
  const int64_t M = tn ? q.n : q.m, K = tn ? q.m : q.n;
  if (pl->bf16) {
    const uint16_t *Ab = static_cast<const uint16_t *>(A);
    float *xt = w.at<float>(pl->off_xt);
    const int ks = gemm_bf16_choose_ksplit(M, K, tn, pl->part_splits(M));
    return tn ? launch_gemm_bf16_tn_main(Ab, q.lda, X, kBld, C, ldc, M, ncols, K, 1.f, 0.f, ks,
                                         part, xt, st)
              : launch_gemm_bf16_nn_main(Ab, q.lda, X, kBld, C, ldc, M, ncols, K, 1.f, 0.f, ks,
                                         part, xt, st);
  }
  const float *Af = static_cast<const float *>(A);
  if (pl->split) {
    // FP32 A on the BF16 matrix cores (exact three-term splits of both
    // operands, six term products): the pass is then bound by streaming A,
    // not by the FP32 matrix-core rate
    float *xt = w.at<float>(pl->off_xt);
    const int ks = gemm_f32s_choose_ksplit(M, K, tn, pl->part_splits(M));
    return tn ? launch_gemm_f32s_tn_main(Af, q.lda, X, kBld, C, ldc, M, ncols, K, 1.f, 0.f, ks,
                                         part, xt, st)
              : launch_gemm_f32s_nn_main(Af, q.lda, X, kBld, C, ldc, M, ncols, K, 1.f, 0.f, ks,
                                         part, xt, st);
  }
  // column-major A is A^T row-major: A X is its TN product, A^T T its NN one
  const bool ktn = pl->colmajor ? !tn : tn;
  const int ks = gemm_choose_ksplit(M, K, ktn, pl->part_splits(M));
  return ktn ? launch_gemm_tn_main(Af, q.lda, X, kBld, C, ldc, M, ncols, K, 1.f, 0.f, ks, part, st)
             : launch_gemm_nn_main(Af, q.lda, X, kBld, C, ldc, M, ncols, K, 1.f, 0.f, ks, part, st);
}

// S = A Omega_j (standardized Bernoulli: A B_j - z), m x kBld.
void sketch(const farpca_plan_s *pl, const Ws &w, const void *A, float *S, hipStream_t st) {
  const farpca_params &q = pl->prm;
  float *part = w.at<float>(pl->off_part);
  if (pl->kind == FARPCA_GAUSSIAN) {
    int nsp;
    {
      ProfScope ps(FARPCA_PROF_GEMM_NN, st);
      nsp = a_pass(pl, w, false, A, w.at<float>(pl->off_om), kBld, S, kBld, st);
    }
    launch_gemm_finish(part, nsp, q.m, kBld, S, kBld, 1.f, 0.f, st);
    return;
  }
  const float *z = (pl->kind == FARPCA_STD_BERNOULLI) ? w.at<float>(pl->off_z) : nullptr;
  const float scale = pl->sketch_scale;
  if (pl->colmajor) {
    ProfScope ps(FARPCA_PROF_SKETCH, st);
    launch_sketch_cols(static_cast<const float *>(A), q.lda, q.m, q.n, pl->b,
                       w.at<ChunkEntry>(pl->off_flat), w.at<uint32_t>(pl->off_colcnt), S, scale, z,
                       -1.f, st);
    return;
  }
  const int ns = sketch_choose_split(q.m, q.n);
  if (ns <= 1) {
    ProfScope ps(FARPCA_PROF_SKETCH, st);
    launch_sketch_full(A, pl->bf16, q.lda, q.m, q.n, pl->b, w.at<uint32_t>(pl->off_colptr),
                       w.at<ChunkEntry>(pl->off_ent), S, 1, scale, z, -1.f, st);
  } else {
    {
      ProfScope ps(FARPCA_PROF_SKETCH, st);
      launch_sketch_full(A, pl->bf16, q.lda, q.m, q.n, pl->b, w.at<uint32_t>(pl->off_colptr),
                         w.at<ChunkEntry>(pl->off_ent), part, ns, scale, z, -1.f, st);
    }
    // number of splits actually launched
    const int64_t nchunks = pl->nchunks;
    const int64_t cps = (nchunks + ns - 1) / ns;
    const int nsp = (int)((nchunks + cps - 1) / cps);
    launch_reduce_partials(part, nsp, q.m, kBld, S, kBld, scale, 0.f, nullptr, 0, 0.f, z, -1.f, st);
  }
}

// T <- (I - Q Q^T) T, applied `passes` times (block classical Gram-Schmidt,
// twice for reorthogonalisation), Q = first l columns of the basis.
void project_out(const farpca_plan_s *pl, const Ws &w, int64_t l, float *T, int passes, hipStream_t st) {
  if (l == 0) return;
  const farpca_params &q = pl->prm;
  float *Q = w.at<float>(pl->off_q);
  float *r = w.at<float>(pl->off_r);
  float *part = w.at<float>(pl->off_part);
  for (int pass = 0; pass < passes; ++pass) {
    launch_gemm_tn(Q, pl->ldq, T, kBld, r, kBld, l, pl->b, q.m, 1.f, 0.f,
                   gemm_choose_ksplit(l, q.m, 1, pl->part_splits(l)), part, st);
    launch_gemm_nn(Q, pl->ldq, r, kBld, T, kBld, q.m, pl->b, l, -1.f, 1.f, 1, part, st);
  }
}

// X (K x b) <- orthonormal basis of its range, CholeskyQR passes
// first_pass .. end_pass - 1 (FP64 Gram and factor, FP32 storage); numerically dependent columns
// (residual below 1e-5 of the column, i.e. rounding noise of the FP32 data)
// become exactly zero.  Two passes suffice: the first leaves an orthogonality
// error of about u64 cond(X)^2, the second brings it to the FP32 rounding of
// the stored result, which further passes cannot go below.  A repeated pass
// whose Gram shows the columns orthonormal to kRepeatSkip already (well
// conditioned X: the first pass reached that level) applies nothing: its
// factor and solve are skipped on the device.  If gram_eig, the eigenvalues of
// the first Gram go to w64 (descending).
void cholqr(const farpca_plan_s *pl, const Ws &w, float *X, int64_t K, int first_pass, int end_pass,
            bool gram_eig, hipStream_t st) {
  double *gpart = w.at<double>(pl->off_gpart);
  double *G = w.at<double>(pl->off_g64);
  double *Rf = w.at<double>(pl->off_rinv);
  int *flags = reinterpret_cast<int *>(w.at<double>(pl->off_scal) + 3);
  int *apply = flags + 1;
  for (int pass = first_pass; pass < end_pass; ++pass) {
    launch_gram(X, kBld, K, pl->b, gpart, G, st);
    if (pass == 0 && gram_eig)
      launch_eig_small(G, pl->b, kMaxBlock, w.at<double>(pl->off_w64), w.at<double>(pl->off_v64),
                       kMaxBlock, st);
    const bool repeat = pass > 0;
    launch_chol(G, pl->b, kDropRel, Rf, flags, repeat ? kRepeatSkip : 0.0, repeat ? apply : nullptr, st);
    launch_trsm_rows(X, kBld, K, pl->b, Rf, X, kBld, repeat ? apply : nullptr, st);
  }
}

}  // namespace

// Step a0 on a workspace that is either full (cap < 0: every block and the
// final part) or a loop part with room for cap blocks.
static int begin_impl(farpca_plan_s *pl, const void *dA, void *dWork, size_t work_bytes,
                      int64_t cap, double *dEhist, hipStream_t st) {
  if (pl->step_pending) {            // a pending block of an abandoned run
    hipEventSynchronize(pl->ev_step);
    pl->step_pending = false;
  }
  pl->stage = 0;
  if ((reinterpret_cast<uintptr_t>(dWork) & 255) != 0) return FARPCA_E_INVALID;
  if (cap < 0) {
    carve_full(pl);
    if (work_bytes < pl->total) return FARPCA_E_NOMEM;
  } else {
    if (cap < 1 || cap > pl->maxblk) return FARPCA_E_INVALID;
    if (work_bytes < carve_loop(pl, cap)) return FARPCA_E_NOMEM;
  }
  const farpca_params &q = pl->prm;
  Ws w{static_cast<char *>(dWork)};
  double *scal = w.at<double>(pl->off_scal);
  double *nA2 = scal + 0, *E = scal + 1;
  int *flags = reinterpret_cast<int *>(scal + 3);

  HIP_OK(hipMemsetAsync(scal, 0, 64, st));
  // a0: ||A||_F^2 in FP64, row sums (z for the standardized Bernoulli matrix), finiteness.
  setup_pass(pl, w, dA, flags, st);
  launch_sum_partials(w.at<double>(pl->off_setup), setup_partials(pl), nA2, st);
  double h_scal[4];
  HIP_OK(hipMemcpyAsync(h_scal, scal, 32, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  int h_flags = 0;
  std::memcpy(&h_flags, &h_scal[3], sizeof(int));
  if (h_flags & 2) return FARPCA_E_NONFINITE;
  HIP_OK(hipMemcpyAsync(E, nA2, 8, hipMemcpyDeviceToDevice, st));
  if (pl->kind == FARPCA_STD_BERNOULLI)
    launch_scale_rowsum(w.at<double>(pl->off_rowsum), q.m, pl->p, w.at<float>(pl->off_z), st);
  pl->run_a = dA;
  pl->run_work = static_cast<char *>(dWork);
  pl->run_work_bytes = work_bytes;
  pl->run_final = cap < 0 ? pl->run_work + pl->off_final : nullptr;
  pl->own_ehist = dEhist == nullptr;
  pl->run_ehist = dEhist ? dEhist : w.at<double>(pl->off_ehist);
  pl->norm_a2 = h_scal[0];
  pl->stop_thr = q.tol * q.tol * pl->norm_a2;
  pl->l = 0;
  pl->blocks = 0;
  pl->status = FARPCA_NOT_CONVERGED;
  pl->stage = 1;
  return FARPCA_OK;
}

extern "C" int farpca_begin(farpca_plan_t *plan, const void *dA, void *dWork, size_t work_bytes,
                            double *dEhist, void *stream) {
  if (!plan || !dA || !dWork) return FARPCA_E_INVALID;
  return begin_impl(plan, dA, dWork, work_bytes, -1, dEhist, static_cast<hipStream_t>(stream));
}

extern "C" size_t farpca_loop_bytes(farpca_plan_t *plan, int64_t cap_blocks) {
  if (!plan || cap_blocks < 1 || cap_blocks > plan->maxblk) return 0;
  // sizing only: the layout of a running solve is left as it is
  farpca_plan_s probe = *plan;
  probe.h_e = nullptr;
  probe.ev_step = nullptr;
  return carve_loop(&probe, cap_blocks);
}

extern "C" int farpca_begin_loop(farpca_plan_t *plan, const void *dA, void *dLoop, size_t bytes,
                                 int64_t cap_blocks, double *dEhist, void *stream) {
  if (!plan || !dA || !dLoop) return FARPCA_E_INVALID;
  if (cap_blocks < 1 || cap_blocks > plan->maxblk) return FARPCA_E_INVALID;
  return begin_impl(plan, dA, dLoop, bytes, cap_blocks, dEhist, static_cast<hipStream_t>(stream));
}

extern "C" int farpca_grow(farpca_plan_t *plan, void *dLoop, size_t bytes, int64_t cap_blocks,
                           void *stream) {
  if (!plan || !dLoop) return FARPCA_E_INVALID;
  farpca_plan_s *pl = plan;
  if (pl->stage != 1 || pl->step_pending || pl->run_final) return FARPCA_E_INVALID;
  if (cap_blocks < pl->cap || cap_blocks > pl->maxblk) return FARPCA_E_INVALID;
  if ((reinterpret_cast<uintptr_t>(dLoop) & 255) != 0) return FARPCA_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const farpca_params &q = pl->prm;
  // offsets of the current layout, then the new one
  farpca_plan_s old = *pl;
  old.h_e = nullptr;
  old.ev_step = nullptr;
  if (bytes < carve_loop(pl, cap_blocks)) {
    carve_loop(pl, old.cap);
    return FARPCA_E_NOMEM;
  }
  Ws wo{pl->run_work}, wn{static_cast<char *>(dLoop)};
  const int64_t l = pl->l;
  // the state the block loop carries: Q and C^T (l columns each), the
  // scalars (||A||^2, E, alpha, flags), the row sums z, the E history
  if (l > 0) {
    HIP_OK(hipMemcpy2DAsync(wn.at<float>(pl->off_q), pl->ldq * 4, wo.at<float>(old.off_q), old.ldq * 4,
                            l * 4, q.m, hipMemcpyDeviceToDevice, st));
    HIP_OK(hipMemcpy2DAsync(wn.at<float>(pl->off_ct), pl->ldq * 4, wo.at<float>(old.off_ct),
                            old.ldq * 4, l * 4, q.n, hipMemcpyDeviceToDevice, st));
  }
  HIP_OK(hipMemcpyAsync(wn.at<char>(pl->off_scal), wo.at<char>(old.off_scal), 64,
                        hipMemcpyDeviceToDevice, st));
  if (pl->kind == FARPCA_STD_BERNOULLI)
    HIP_OK(hipMemcpyAsync(wn.at<char>(pl->off_z), wo.at<char>(old.off_z), (size_t)q.m * 4,
                          hipMemcpyDeviceToDevice, st));
  if (pl->own_ehist) {
    HIP_OK(hipMemcpyAsync(wn.at<char>(pl->off_ehist), wo.at<char>(old.off_ehist),
                          (size_t)pl->maxblk * 8, hipMemcpyDeviceToDevice, st));
    pl->run_ehist = wn.at<double>(pl->off_ehist);
  }
  pl->run_work = static_cast<char *>(dLoop);
  pl->run_work_bytes = bytes;
  return FARPCA_OK;
}

// One block of the method (Algorithm 1/2: test matrix, sketch, power steps,
// basis extension, indicator update), enqueued on `st`, followed by an
// asynchronous read-back of E into pinned host memory and an event.
static int enqueue_block(farpca_plan_s *pl, hipStream_t st) {
  const farpca_params &q = pl->prm;
  const int64_t m = q.m, n = q.n;
  const int b = pl->b;
  const void *A = pl->run_a;
  Ws w{pl->run_work};
  double *scal = w.at<double>(pl->off_scal);
  double *E = scal + 1, *alpha = scal + 2;
  float *Q = w.at<float>(pl->off_q);
  float *Ct = w.at<float>(pl->off_ct);
  float *S = w.at<float>(pl->off_s);
  float *Yb = w.at<float>(pl->off_y);
  float *X = w.at<float>(pl->off_x);
  float *part = w.at<float>(pl->off_part);
  const int64_t j = pl->blocks;
  int64_t l = pl->l;
  if (l + b > pl->cap * b) return FARPCA_E_NOMEM;   // grow the loop part first
  if (!pl->h_e) {
    void *h = nullptr;
    HIP_OK(hipHostMalloc(&h, 64, hipHostMallocDefault));
    pl->h_e = static_cast<double *>(h);
  }
  if (!pl->ev_step) HIP_OK(hipEventCreateWithFlags(&pl->ev_step, hipEventDisableTiming));

  gen_omega(pl, w, j, st);
  sketch(pl, w, A, S, st);
  float *Ysrc = S;
  if (pl->P > 0) {
    float *G = w.at<float>(pl->off_g);
    HIP_OK(hipMemsetAsync(alpha, 0, 8, st));
    float *T = S;
    for (int k = 1; k <= pl->P; ++k) {
      project_out(pl, w, l, T, 2, st);
      int nsp;
      {
        ProfScope ps(FARPCA_PROF_GEMM_TN, st);
        nsp = a_pass(pl, w, true, A, T, b, X, kBld, st);
      }
      launch_gemm_finish(part, nsp, n, b, X, kBld, 1.f, 0.f, st);
      if (k >= 2 && pl->P > 2) launch_axpy_block(X, kBld, G, kBld, n, b, alpha, st);
      cholqr(pl, w, X, n, 0, kCholqrPasses, pl->P > 2, st);
      if (k >= 2 && pl->P > 2) launch_alpha_update(w.at<double>(pl->off_w64), b, alpha, st);
      launch_copy_block(X, kBld, n, b, G, kBld, st);
      if (k < pl->P) {
        int nsp2;
        {
          ProfScope ps(FARPCA_PROF_GEMM_NN, st);
          nsp2 = a_pass(pl, w, false, A, G, b, S, kBld, st);
        }
        launch_gemm_finish(part, nsp2, m, b, S, kBld, 1.f, 0.f, st);
        T = S;
      }
    }
    int nsp3;
    {
      ProfScope ps(FARPCA_PROF_GEMM_NN, st);
      nsp3 = a_pass(pl, w, false, A, G, b, Yb, kBld, st);
    }
    launch_gemm_finish(part, nsp3, m, b, Yb, kBld, 1.f, 0.f, st);
    Ysrc = Yb;
  }
  // Basis extension: Y_j against Q, orthonormalise, append; C_j^T = A^T Q_j.
  // The first CholeskyQR pass multiplies by R^{-1}, which magnifies what the
  // projections leave of span(Q) (FP32 rounding, about u ||Y_j||) by up to
  // cond(Y_j): for blocks that fall almost inside span(Q) (sparse test
  // matrices on a matrix whose right singular vectors are sparse, Section
  // 5.5) that reaches 1e-3..1e-2, Q loses orthogonality and the indicator
  // counts directions twice.  One more projection after that pass removes the
  // magnified part; the second pass restores unit columns.
  project_out(pl, w, l, Ysrc, 2, st);
  cholqr(pl, w, Ysrc, m, 0, 1, false, st);
  project_out(pl, w, l, Ysrc, 1, st);
  cholqr(pl, w, Ysrc, m, 1, kCholqrPasses, false, st);
  launch_copy_block(Ysrc, kBld, m, b, Q + l, pl->ldq, st);
  if (pl->c64) {
    // small tol: the indicator needs ||C_j||^2 below the FP32 accumulation error
    const int ns64 = cpass64_choose_split(n, m, pl->part_floats / 2 / (n * kBld));
    launch_cpass64(A, pl->bf16, pl->colmajor, q.lda, Ysrc, kBld, n, m, b, ns64,
                   reinterpret_cast<double *>(part), Ct + l, pl->ldq, w.at<double>(pl->off_sq), st);
  } else {
    int nsp4;
    {
      ProfScope ps(FARPCA_PROF_GEMM_C, st);
      nsp4 = a_pass(pl, w, true, A, Ysrc, b, Ct + l, pl->ldq, st);
    }
    launch_gemm_finish(part, nsp4, n, b, Ct + l, pl->ldq, 1.f, 0.f, st);
    launch_sqnorm(Ct + l, pl->ldq, n, b, w.at<double>(pl->off_sq), st);
  }
  launch_indicator_update(w.at<double>(pl->off_sq), sqnorm_num_partials(n), E, pl->run_ehist, j,
                          st);
  l += b;
  pl->l = l;
  pl->blocks = (int)(j + 1);
  HIP_OK(hipMemcpyAsync(pl->h_e, E, 8, hipMemcpyDeviceToHost, st));
  HIP_OK(hipEventRecord(pl->ev_step, st));
  return FARPCA_OK;
}

extern "C" int farpca_step_async(farpca_plan_t *plan, void *stream) {
  if (!plan) return FARPCA_E_INVALID;
  farpca_plan_s *pl = plan;
  if (pl->stage == 2 && !pl->step_pending) return 0;
  if (pl->stage != 1 || pl->step_pending) return FARPCA_E_INVALID;
  const int rc = enqueue_block(pl, static_cast<hipStream_t>(stream));
  if (rc != FARPCA_OK) return rc;
  pl->step_pending = true;
  return 1;
}

extern "C" int farpca_step_poll(farpca_plan_t *plan, int wait) {
  if (!plan) return FARPCA_E_INVALID;
  farpca_plan_s *pl = plan;
  if (!pl->step_pending) return pl->stage == 2 ? 0 : (pl->stage == 1 ? 1 : FARPCA_E_INVALID);
  if (wait) {
    HIP_OK(hipEventSynchronize(pl->ev_step));
  } else {
    const hipError_t e = hipEventQuery(pl->ev_step);
    if (e == hipErrorNotReady) return 2;
    if (e != hipSuccess) return FARPCA_E_DEVICE;
  }
  pl->step_pending = false;
  const double e_host = *pl->h_e;
  bool done = false;
  if (pl->prm.rank > 0) {
    if (pl->l >= pl->prm.rank) done = true;
  } else if (e_host < pl->stop_thr) {
    done = true;
  }
  if (done) pl->status = FARPCA_OK;
  if (done || pl->blocks >= pl->maxblk) {
    pl->stage = 2;
    return 0;
  }
  return 1;
}

extern "C" int farpca_step(farpca_plan_t *plan, void *stream) {
  const int rc = farpca_step_async(plan, stream);
  if (rc != 1) return rc;
  return farpca_step_poll(plan, 1);
}


// Step a10 with the final part at dFinal (sized for the reached l) and the
// outputs U (m x ldu), S, V (n x ldv).
static int finish_impl(farpca_plan_s *pl, char *dFinal, void *dU, int64_t ldu, double *dS,
                       void *dV, int64_t ldv, farpca_info *info, hipStream_t st) {
  const farpca_params &q = pl->prm;
  const int64_t m = q.m, n = q.n;
  Ws w{pl->run_work};
  double *scal = w.at<double>(pl->off_scal);
  float *Q = w.at<float>(pl->off_q);
  float *Ct = w.at<float>(pl->off_ct);
  float *part = w.at<float>(pl->off_part);
  const int64_t l = pl->l;
  const int status = pl->status;
  // the final part is laid out for l columns (for l_max inside a full workspace)
  const FinalLayout fl = final_layout(n, pl->run_final ? pl->lmax : l);
  Ws wf{dFinal};

  // Final decomposition: K = C C^T = (C^T)^T C^T, eigenpairs descending.
  const int64_t rout = (q.rank > 0) ? imin(q.rank, l) : l;
  double *Kbig = wf.at<double>(fl.kbig);
  double *wfin = wf.at<double>(fl.wfin);
  double *vfin = wf.at<double>(fl.vfin);
  float *u32 = wf.at<float>(fl.u32);
  launch_gram_big(Ct, pl->ldq, n, l, Kbig, wf.at<void>(fl.gbig), fl.gbig_bytes, st);
  int sweeps;
  bool eig_ok = false;
  {
    ProfScope ps(FARPCA_PROF_EIG, st);
    sweeps = eig_sym(Kbig, l, wfin, vfin, wf.at<void>(fl.eig), kFinalEigRel, st, &eig_ok);
  }
  launch_sqrt_clip(wfin, rout, dS, st);
  launch_trunc_rank(dS, rout, scal, q.tol, q.rank > 0, reinterpret_cast<int64_t *>(scal + 4), st);
  // U = Q U~ (first rout columns)
  launch_convert_f64_f32(vfin, l, rout, l, nullptr, u32, rout, st);
  for (int64_t c0 = 0; c0 < rout; c0 += kBld) {
    const int64_t nc = imin(kBld, rout - c0);
    launch_gemm_nn(Q, pl->ldq, u32 + c0, rout, static_cast<float *>(dU) + c0, ldu, m, nc, l,
                   1.f, 0.f, 1, part, st);
  }
  // V = C^T U~ Sigma^{-1}
  launch_convert_f64_f32(vfin, l, rout, l, dS, u32, rout, st);
  for (int64_t c0 = 0; c0 < rout; c0 += kBld) {
    const int64_t nc = imin(kBld, rout - c0);
    launch_gemm_nn(Ct, pl->ldq, u32 + c0, rout, static_cast<float *>(dV) + c0, ldv, n, nc, l,
                   1.f, 0.f, 1, part, st);
  }
  double h_tail[5];
  HIP_OK(hipMemcpyAsync(h_tail, scal, 40, hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  HIP_OK(hipGetLastError());
  if (g_prof.on) prof_resolve();
  pl->stage = 0;
  if (info) {
    info->rank_l = l;
    info->rank_out = rout;
    info->blocks = pl->blocks;
    info->status = status;
    info->norm_a2 = pl->norm_a2;
    info->err_indicator = h_tail[1];
    info->eig_sweeps = sweeps;
    int fg = 0;
    std::memcpy(&fg, &h_tail[3], sizeof(int));
    std::memcpy(&info->rank_trunc, &h_tail[4], sizeof(int64_t));
    info->dropped = fg & 1;
    info->eig_converged = eig_ok ? 1 : 0;
    info->reserved1 = 0;
  }
  return status;
}

extern "C" int farpca_finish(farpca_plan_t *plan, void *dU, double *dS, void *dV,
                             farpca_info *info, void *stream) {
  if (!plan || !dU || !dS || !dV) return FARPCA_E_INVALID;
  farpca_plan_s *pl = plan;
  if (pl->stage == 0 || pl->blocks == 0 || pl->step_pending || !pl->run_final)
    return FARPCA_E_INVALID;
  return finish_impl(pl, pl->run_final, dU, pl->lmax, dS, dV, pl->lmax, info,
                     static_cast<hipStream_t>(stream));
}

extern "C" size_t farpca_final_bytes(farpca_plan_t *plan) {
  if (!plan || plan->blocks == 0) return 0;
  return final_layout(plan->prm.n, plan->l).total;
}

extern "C" int farpca_finish_final(farpca_plan_t *plan, void *dFinal, size_t bytes, void *dU,
                                   int64_t ldu, double *dS, void *dV, int64_t ldv,
                                   farpca_info *info, void *stream) {
  if (!plan || !dFinal || !dU || !dS || !dV) return FARPCA_E_INVALID;
  farpca_plan_s *pl = plan;
  if (pl->stage == 0 || pl->blocks == 0 || pl->step_pending) return FARPCA_E_INVALID;
  if ((reinterpret_cast<uintptr_t>(dFinal) & 255) != 0) return FARPCA_E_INVALID;
  const int64_t rout = (pl->prm.rank > 0) ? imin(pl->prm.rank, pl->l) : pl->l;
  if (ldu < rout || ldv < rout) return FARPCA_E_INVALID;
  if (bytes < final_layout(pl->prm.n, pl->l).total) return FARPCA_E_NOMEM;
  pl->run_final = nullptr;             // laid out for the reached l
  return finish_impl(pl, static_cast<char *>(dFinal), dU, ldu, dS, dV, ldv, info,
                     static_cast<hipStream_t>(stream));
}

extern "C" int farpca_run(farpca_plan_t *plan, const void *dA, void *dWork, size_t work_bytes,
                          void *dU, double *dS, void *dV, farpca_info *info, double *dEhist,
                          void *stream) {
  if (!plan || !dA || !dWork || !dU || !dS || !dV) return FARPCA_E_INVALID;
  int rc = farpca_begin(plan, dA, dWork, work_bytes, dEhist, stream);
  if (rc != FARPCA_OK) return rc;
  while ((rc = farpca_step(plan, stream)) == 1) {
  }
  if (rc < 0) {
    plan->stage = 0;
    return rc;
  }
  return farpca_finish(plan, dU, dS, dV, info, stream);
}

// ---- the run without a caller workspace (callers that cannot allocate)
//
// `scratch` is the workspace of farpca_run_static: a file-scope device array
// that every GPU the library runs on holds from module load until the process
// ends.  In host code its name is only a stand-in for the symbol; the device
// address comes from hipGetSymbolAddress, once per device (with that device
// current), and only that address is passed on.  Every call on one GPU shares
// the array: runs that overlap on one GPU race, and a run may leave anything
// in it (farpca_run clears what it needs at the start).
static __device__ __align__(256) char scratch[FARPCA_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (nullptr on a HIP error).
void *static_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" int farpca_run_static(farpca_plan_t *plan, const void *dA, void *dU, double *dS,
                                 void *dV, farpca_info *info, double *dEhist, void *stream) {
  if (!plan || !dA || !dU || !dS || !dV) return FARPCA_E_INVALID;
  if (plan->total > (size_t)FARPCA_STATIC_SCRATCH_BYTES) return FARPCA_E_NOMEM;
  void *ws = static_scratch();
  if (!ws) return FARPCA_E_DEVICE;
  return farpca_run(plan, dA, ws, (size_t)FARPCA_STATIC_SCRATCH_BYTES, dU, dS, dV, info, dEhist,
                    stream);
}

extern "C" int farpca_omega(farpca_plan_t *plan, int64_t block_j, void *dWork, size_t work_bytes,
                            uint64_t *dMask, uint64_t *dNeg, float *dDense, void *stream) {
  if (!plan || !dWork || !dMask || !dNeg || !dDense || block_j < 0) return FARPCA_E_INVALID;
  // the workspace of a run between farpca_begin and farpca_finish is in use
  if (plan->stage != 0) return FARPCA_E_INVALID;
  carve_full(plan);
  if (work_bytes < plan->total) return FARPCA_E_NOMEM;
  Ws w{static_cast<char *>(dWork)};
  hipStream_t st = static_cast<hipStream_t>(stream);
  gen_omega(plan, w, block_j, st, dMask, dNeg, dDense);
  HIP_OK(hipGetLastError());
  return FARPCA_OK;
}

extern "C" int farpca_sketch(farpca_plan_t *plan, const void *dA, int64_t block_j, void *dWork,
                             size_t work_bytes, float *dS, void *stream) {
  if (!plan || !dA || !dWork || !dS || block_j < 0) return FARPCA_E_INVALID;
  if (plan->stage != 0) return FARPCA_E_INVALID;     // workspace held by a run
  carve_full(plan);
  if (work_bytes < plan->total) return FARPCA_E_NOMEM;
  if ((reinterpret_cast<uintptr_t>(dWork) & 255) != 0) return FARPCA_E_INVALID;
  farpca_plan_s *pl = plan;
  Ws w{static_cast<char *>(dWork)};
  hipStream_t st = static_cast<hipStream_t>(stream);
  const farpca_params &q = pl->prm;
  // the setup pass of the run (finiteness flag; row sums for the standardized
  // Bernoulli matrix): a sketch of A with NaN / Inf is rejected as by farpca_begin
  double *scal = w.at<double>(pl->off_scal);
  int *flags = reinterpret_cast<int *>(scal + 3);
  HIP_OK(hipMemsetAsync(scal, 0, 64, st));
  setup_pass(pl, w, dA, flags, st);
  int h_flags = 0;
  HIP_OK(hipMemcpyAsync(&h_flags, flags, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  if (h_flags & 2) return FARPCA_E_NONFINITE;
  if (pl->kind == FARPCA_STD_BERNOULLI)
    launch_scale_rowsum(w.at<double>(pl->off_rowsum), q.m, pl->p, w.at<float>(pl->off_z), st);
  gen_omega(pl, w, block_j, st);
  sketch(pl, w, dA, dS, st);
  HIP_OK(hipGetLastError());
  return FARPCA_OK;
}

extern "C" size_t farpca_gemm_scratch_bytes(int64_t M) { return (size_t)16 * M * kBld * 4; }

extern "C" int farpca_gemm_nn(const float *dA, int64_t lda, const float *dX, int64_t ldx, float *dC,
                              int64_t ldc, int64_t M, int64_t N, int64_t K, float *dPart,
                              void *stream) {
  if (!dA || !dX || !dC || M < 1 || K < 1 || N < 1 || N > kBld || lda < K || ldx < N || ldc < N)
    return FARPCA_E_INVALID;
  const int ks = gemm_choose_ksplit(M, K, 0, 16);
  if (ks > 1 && !dPart) return FARPCA_E_INVALID;
  launch_gemm_nn(dA, lda, dX, ldx, dC, ldc, M, N, K, 1.f, 0.f, ks, dPart,
                 static_cast<hipStream_t>(stream));
  HIP_OK(hipGetLastError());
  return FARPCA_OK;
}

extern "C" int farpca_gemm_tn(const float *dA, int64_t lda, const float *dY, int64_t ldy, float *dC,
                              int64_t ldc, int64_t M, int64_t N, int64_t K, float *dPart,
                              void *stream) {
  if (!dA || !dY || !dC || M < 1 || K < 1 || N < 1 || N > kBld || lda < M || ldy < N || ldc < N)
    return FARPCA_E_INVALID;
  const int ks = gemm_choose_ksplit(M, K, 1, 16);
  if (ks > 1 && !dPart) return FARPCA_E_INVALID;
  launch_gemm_tn(dA, lda, dY, ldy, dC, ldc, M, N, K, 1.f, 0.f, ks, dPart,
                 static_cast<hipStream_t>(stream));
  HIP_OK(hipGetLastError());
  return FARPCA_OK;
}

extern "C" size_t farpca_gemm_bf16_scratch_bytes(int64_t M, int64_t K) {
  if (M < 1 || K < 1) return 0;
  return align_up((size_t)16 * M * kBld * 4) + bf16_pack_bytes(K);
}

extern "C" int farpca_gemm_bf16_nn(const uint16_t *dA, int64_t lda, const float *dX, int64_t ldx,
                                   float *dC, int64_t ldc, int64_t M, int64_t N, int64_t K,
                                   void *dScratch, void *stream) {
  if (!dA || !dX || !dC || !dScratch || M < 1 || K < 1 || N < 1 || N > kBld || lda < K ||
      ldx < N || ldc < N)
    return FARPCA_E_INVALID;
  if ((reinterpret_cast<uintptr_t>(dScratch) & 255) != 0) return FARPCA_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float *part = static_cast<float *>(dScratch);
  float *xt = reinterpret_cast<float *>(static_cast<char *>(dScratch) +
                                        align_up((size_t)16 * M * kBld * 4));
  const int ks = gemm_bf16_choose_ksplit(M, K, 0, 16);
  const int nsp = launch_gemm_bf16_nn_main(dA, lda, dX, ldx, dC, ldc, M, N, K, 1.f, 0.f, ks, part,
                                           xt, st);
  launch_gemm_finish(part, nsp, M, N, dC, ldc, 1.f, 0.f, st);
  HIP_OK(hipGetLastError());
  return FARPCA_OK;
}

extern "C" int farpca_gemm_bf16_tn(const uint16_t *dA, int64_t lda, const float *dY, int64_t ldy,
                                   float *dC, int64_t ldc, int64_t M, int64_t N, int64_t K,
                                   void *dScratch, void *stream) {
  if (!dA || !dY || !dC || !dScratch || M < 1 || K < 1 || N < 1 || N > kBld || lda < M ||
      ldy < N || ldc < N)
    return FARPCA_E_INVALID;
  if ((reinterpret_cast<uintptr_t>(dScratch) & 255) != 0) return FARPCA_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float *part = static_cast<float *>(dScratch);
  float *xt = reinterpret_cast<float *>(static_cast<char *>(dScratch) +
                                        align_up((size_t)16 * M * kBld * 4));
  const int ks = gemm_bf16_choose_ksplit(M, K, 1, 16);
  const int nsp = launch_gemm_bf16_tn_main(dA, lda, dY, ldy, dC, ldc, M, N, K, 1.f, 0.f, ks, part,
                                           xt, st);
  launch_gemm_finish(part, nsp, M, N, dC, ldc, 1.f, 0.f, st);
  HIP_OK(hipGetLastError());
  return FARPCA_OK;
}

extern "C" int farpca_gemm_f32s_nn(const float *dA, int64_t lda, const float *dX, int64_t ldx,
                                   float *dC, int64_t ldc, int64_t M, int64_t N, int64_t K,
                                   void *dScratch, void *stream) {
  if (!dA || !dX || !dC || !dScratch || M < 1 || K < 1 || N < 1 || N > kBld || lda < K ||
      ldx < N || ldc < N)
    return FARPCA_E_INVALID;
  if ((reinterpret_cast<uintptr_t>(dScratch) & 255) != 0) return FARPCA_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float *part = static_cast<float *>(dScratch);
  float *xt = reinterpret_cast<float *>(static_cast<char *>(dScratch) +
                                        align_up((size_t)16 * M * kBld * 4));
  const int ks = gemm_f32s_choose_ksplit(M, K, 0, 16);
  const int nsp = launch_gemm_f32s_nn_main(dA, lda, dX, ldx, dC, ldc, M, N, K, 1.f, 0.f, ks, part,
                                           xt, st);
  launch_gemm_finish(part, nsp, M, N, dC, ldc, 1.f, 0.f, st);
  HIP_OK(hipGetLastError());
  return FARPCA_OK;
}

extern "C" int farpca_gemm_f32s_tn(const float *dA, int64_t lda, const float *dY, int64_t ldy,
                                   float *dC, int64_t ldc, int64_t M, int64_t N, int64_t K,
                                   void *dScratch, void *stream) {
  if (!dA || !dY || !dC || !dScratch || M < 1 || K < 1 || N < 1 || N > kBld || lda < M ||
      ldy < N || ldc < N)
    return FARPCA_E_INVALID;
  if ((reinterpret_cast<uintptr_t>(dScratch) & 255) != 0) return FARPCA_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  float *part = static_cast<float *>(dScratch);
  float *xt = reinterpret_cast<float *>(static_cast<char *>(dScratch) +
                                        align_up((size_t)16 * M * kBld * 4));
  const int ks = gemm_f32s_choose_ksplit(M, K, 1, 16);
  const int nsp = launch_gemm_f32s_tn_main(dA, lda, dY, ldy, dC, ldc, M, N, K, 1.f, 0.f, ks, part,
                                           xt, st);
  launch_gemm_finish(part, nsp, M, N, dC, ldc, 1.f, 0.f, st);
  HIP_OK(hipGetLastError());
  return FARPCA_OK;
}

extern "C" size_t farpca_eig_scratch_bytes(int64_t l) { return eig_workspace_bytes(l); }

extern "C" int farpca_eig(const double *dK, int64_t l, double *dW, double *dV, void *dWork,
                          double rel, int *converged, void *stream) {
  if (!dK || !dW || !dV || !dWork || l < 1 || !(rel < 1.0)) return FARPCA_E_INVALID;
  bool ok = false;
  const int sweeps = eig_sym(dK, l, dW, dV, dWork, rel, static_cast<hipStream_t>(stream), &ok);
  HIP_OK(hipGetLastError());
  if (converged) *converged = ok ? 1 : 0;
  return sweeps;
}

extern "C" void farpca_profile_enable(int on) {
  if (!on && g_prof.npend) prof_resolve();
  g_prof.on = on != 0;
  if (on) {
    for (auto &c : g_prof.cls) c = ProfClass();
  }
}

extern "C" int farpca_profile_get(int cls, double *total_ms, int64_t *count) {
  if (cls < 0 || cls >= FARPCA_PROF_NCLASS || !total_ms || !count) return FARPCA_E_INVALID;
  *total_ms = g_prof.cls[cls].total_ms;
  *count = g_prof.cls[cls].count;
  return FARPCA_OK;
}
