// FP64 symmetric eigensolver for the final small decomposition of the method
// (Algorithm 1/2 final steps: the eigendecomposition whose square roots are
// the singular values of C = Q^T A), and for the b x b Gram of the power block
// (smallest singular value for the shift).
//
// Method: two-sided cyclic Jacobi.  Small matrices (<= 64) are solved by one
// workgroup entirely in LDS.  Larger ones are first rotated by (approximate,
// two Jacobi sweeps) eigenvectors of their 64 x 64 diagonal blocks (the
// method builds K = C C^T block by block, and blocks of later power iterations
// couple weakly, so this leaves little off-diagonal mass), then finished by
// block Jacobi: the index set is cut into blocks of 16, blocks are paired by a
// round-robin tournament, every pair's 32 x 32 principal submatrix gets one
// Jacobi sweep in LDS (one workgroup per pair), and the whole matrix is then
// rotated block-by-block,
// M[S_p, S_q] <- R_p^T M[S_p, S_q] R_q, V[:, S_q] <- V[:, S_q] R_q - every
// output block depends only on the same input block, so the update runs in
// place with one workgroup per block.  Sweeps repeat until every off-diagonal
// entry is negligible relative to its diagonal pair.  Padding rows/columns are
// exactly zero and never couple (their rotations are the identity).
#include <cmath>

#include "internal.h"

namespace farpca_int {

// A pair (p, q) is left alone when |a_pq| <= rel sqrt(|a_pp a_qq|) (the
// relative test that keeps Jacobi's small eigenvalues accurate; rel = 1e-14
// unless the caller asks for less) or when
// |a_pq| <= 1e-13 max_i |a_ii|.  The absolute floor sits above the FP64
// rounding that the block updates themselves leave behind (sums of 32 terms
// of size max |a_ii|); with a floor at that level the sweeps never end.
constexpr double kJacobiRel = 1e-14;
constexpr double kJacobiAbs = 1e-13;
constexpr int kInnerMaxSweeps = 30;   // a small matrix solved on its own
// Inside the block method a diagonal-block pre-rotation and a pair subproblem
// need not be converged: each is one step of the outer iteration, whose own
// test decides convergence.  (One inner sweep per pair costs about one more
// outer sweep than solving every pair exactly, at a small fraction of the work.)
constexpr int kPreSweeps = 2;
constexpr int kPairSweeps = 1;

__device__ __forceinline__ bool negligible(double apq, double app, double aqq, double floor_abs,
                                           double rel) {
  const double x = fabs(apq);
  return x == 0.0 || x <= rel * sqrt(fabs(app) * fabs(aqq)) || x <= floor_abs;
}

__device__ __forceinline__ int rr_player(int pos, int step, int n) {
  // circle method: position 0 fixed, the others rotate
  return pos == 0 ? 0 : ((pos - 1 + step) % (n - 1)) + 1;
}

// Rotation that (nearly) zeroes a_pq: t = tan(angle) from the hardware
// reciprocal and square root (a few ulps off the exact angle, which only
// leaves a tiny a_pq for the next sweep), then c = 1 / sqrt(1 + t^2) to full
// FP64 accuracy (hardware reciprocal square root and one Newton step) and
// s = t c, so that c^2 + s^2 = 1 to rounding and every update below is an
// exact similarity.  Standard form: theta = (a_qq - a_pp) / (2 a_pq),
// t = sign(theta) / (|theta| + sqrt(theta^2 + 1)); here multiplied through
// by |2 a_pq|: t = sign(d) 2 a_pq / (|d| + sqrt(d^2 + 4 a_pq^2)), d = a_qq - a_pp,
// with d and 2 a_pq first scaled by about 1 / max(|d|, |2 a_pq|) (t depends
// only on their ratio; the squares neither overflow nor underflow).
__device__ __forceinline__ void jacobi_rotation(double app, double aqq, double apq, double &c,
                                                double &s) {
  const double d0 = aqq - app, e0 = 2.0 * apq;
  const double sc = __builtin_amdgcn_rcp(fmax(fabs(d0), fabs(e0)));   // a_pq != 0 here
  const double d = d0 * sc, e = e0 * sc;
  const double h = __builtin_amdgcn_sqrt(fma(d, d, e * e));
  const double t = (d >= 0.0 ? e : -e) * __builtin_amdgcn_rcp(fabs(d) + h);
  const double u = fma(t, t, 1.0);
  double r = __builtin_amdgcn_rsq(u);
  r = r * fma(-0.5 * u * r, r, 1.5);
  c = r;
  s = t * r;
}

// Cyclic Jacobi on an S x S symmetric matrix a (LDS, stride LD) accumulating
// rotations into v (LDS, stride LD, holds the starting orthogonal matrix).
// A step: threads 0 .. S/2 - 1 compute the step's rotations (c, s and
// whether the pair is rotated at all) into LDS; then every thread applies
// them to its 2 x 2 blocks of a (rows, then columns; the diagonal blocks
// like the others) and its row pairs of v.  The pairs of a step follow from
// the step number alone, so the appliers compute them and read the rotation
// together with the matrix entries (one LDS round trip); an identity
// rotation is applied like any other (c = 1, s = 0 copy exactly).
template <int S, int LD, int NT>
__device__ void jacobi_lds(double *a, double *v, double floor_abs, int max_sweeps, double rel) {
  constexpr int H = S / 2;
  __shared__ double cs_c[H], cs_s[H];
  __shared__ int any_rot;
  const int tid = threadIdx.x;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) any_rot = 0;
    __syncthreads();
    for (int step = 0; step < S - 1; ++step) {
      if (tid < H) {
        const int p = rr_player(tid, step, S), q = rr_player(S - 1 - tid, step, S);
        const double app = a[p * LD + p], aqq = a[q * LD + q], apq = a[p * LD + q];
        double c = 1.0, s = 0.0;
        if (!negligible(apq, app, aqq, floor_abs, rel)) {
          jacobi_rotation(app, aqq, apq, c, s);
          any_rot = 1;
        }
        cs_c[tid] = c; cs_s[tid] = s;
      }
      __syncthreads();
      for (int e = tid; e < H * H; e += NT) {
        const int ia = e / H, ib = e % H;
        const int pa = rr_player(ia, step, S), qa = rr_player(S - 1 - ia, step, S);
        const int pb = rr_player(ib, step, S), qb = rr_player(S - 1 - ib, step, S);
        const double ca = cs_c[ia], sa = cs_s[ia], cb = cs_c[ib], sb = cs_s[ib];
        const double x11 = a[pa * LD + pb], x12 = a[pa * LD + qb];
        const double x21 = a[qa * LD + pb], x22 = a[qa * LD + qb];
        const double y11 = ca * x11 - sa * x21, y12 = ca * x12 - sa * x22;
        const double y21 = sa * x11 + ca * x21, y22 = sa * x12 + ca * x22;
        a[pa * LD + pb] = cb * y11 - sb * y12;
        a[pa * LD + qb] = sb * y11 + cb * y12;
        a[qa * LD + pb] = cb * y21 - sb * y22;
        a[qa * LD + qb] = sb * y21 + cb * y22;
      }
      for (int e = tid; e < S * H; e += NT) {
        const int r = e / H, ib = e % H;
        const int pb = rr_player(ib, step, S), qb = rr_player(S - 1 - ib, step, S);
        const double c = cs_c[ib], s = cs_s[ib];
        const double vp = v[r * LD + pb], vq = v[r * LD + qb];
        v[r * LD + pb] = c * vp - s * vq;
        v[r * LD + qb] = s * vp + c * vq;
      }
      __syncthreads();
    }
    if (!any_rot) break;
    __syncthreads();
  }
}

constexpr int kSmallLd = 65;

__global__ __launch_bounds__(256) void eig_small_kernel(const double *__restrict__ K, int s, int ldk,
                                                        double *__restrict__ w, double *__restrict__ V,
                                                        int ldv) {
  __shared__ double a[64 * kSmallLd];
  __shared__ double v[64 * kSmallLd];
  __shared__ double fl;
  __shared__ int perm[64];
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    a[i * kSmallLd + j] = (i < s && j < s) ? K[i * ldk + j] : 0.0;
    v[i * kSmallLd + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < s; ++i) mx = fmax(mx, fabs(a[i * kSmallLd + i]));
    fl = mx * kJacobiAbs;
  }
  __syncthreads();
  jacobi_lds<64, kSmallLd, 256>(a, v, fl, kInnerMaxSweeps, kJacobiRel);
  __syncthreads();
  // descending order among the first s positions (ties by index)
  if (tid < s) {
    const double wi = a[tid * kSmallLd + tid];
    int rank = 0;
    for (int j = 0; j < s; ++j) {
      const double wj = a[j * kSmallLd + j];
      rank += (wj > wi) || (wj == wi && j < tid);
    }
    perm[rank] = tid;
  }
  __syncthreads();
  if (tid < s) w[tid] = a[perm[tid] * kSmallLd + perm[tid]];
  for (int e = tid; e < s * s; e += 256) {
    const int r = e / s, k = e % s;
    V[r * ldv + k] = v[r * kSmallLd + perm[k]];
  }
}

void launch_eig_small(const double *K, int s, int ldk, double *w, double *Vout, int ldv,
                      hipStream_t st) {
  hipLaunchKernelGGL(eig_small_kernel, dim3(1), dim3(256), 0, st, K, s, ldk, w, Vout, ldv);
}

// ------------------------------------------------------------- block Jacobi
constexpr int kBlk = 16;           // block width
constexpr int kSub = 2 * kBlk;     // subproblem size
constexpr int kSubLd = kSub + 1;

__device__ __forceinline__ int sub_index(int u, int bi, int bj) {
  return u < kBlk ? bi * kBlk + u : bj * kBlk + (u - kBlk);
}

// One workgroup per pair: one Jacobi sweep of M[S, S], S = block(bi) U block(bj).
constexpr int kPairThreads = 512;
__global__ __launch_bounds__(kPairThreads) void bj_pair_kernel(const double *__restrict__ M, int64_t lp, int nb,
                                                     int step, double *__restrict__ R,
                                                     const double *__restrict__ floor_abs,
                                                     double rel) {
  __shared__ double a[kSub * kSubLd];
  __shared__ double v[kSub * kSubLd];
  const int pair = blockIdx.x, tid = threadIdx.x;
  const int bi = rr_player(pair, step, nb), bj = rr_player(nb - 1 - pair, step, nb);
  for (int e = tid; e < kSub * kSub; e += kPairThreads) {
    const int u = e / kSub, x = e % kSub;
    a[u * kSubLd + x] = M[(int64_t)sub_index(u, bi, bj) * lp + sub_index(x, bi, bj)];
    v[u * kSubLd + x] = (u == x) ? 1.0 : 0.0;
  }
  __shared__ int any_big;
  if (tid == 0) any_big = 0;
  __syncthreads();
  const double fl = floor_abs[0];
  for (int e = tid; e < kSub * kSub; e += kPairThreads) {
    const int u = e / kSub, x = e % kSub;
    if (u < x && !negligible(a[u * kSubLd + x], a[u * kSubLd + u], a[x * kSubLd + x], fl, rel)) any_big = 1;
  }
  __syncthreads();
  if (any_big) jacobi_lds<kSub, kSubLd, kPairThreads>(a, v, fl, kPairSweeps, rel);   // else R = I
  __syncthreads();
  double *Rp = R + (int64_t)pair * kSub * kSub;
  for (int e = tid; e < kSub * kSub; e += kPairThreads) Rp[e] = v[(e / kSub) * kSubLd + (e % kSub)];
}

// 32 x 32 products on the FP64 matrix cores (v_mfma_f64_16x16x4f64): wave w
// of the workgroup forms the 16 x 16 quadrant (w / 2, w % 2) of L * Rm (L read
// transposed when TRANS_L), K = 32 in 8 steps.  Operand layout: lane l holds
// A (row l % 16, k l / 16) and B (k l / 16, col l % 16); result element v of
// lane l is (row 4 v + l / 16, col l % 16).
typedef double doublex4 __attribute__((ext_vector_type(4)));
template <bool TRANS_L>
__device__ __forceinline__ doublex4 mm32_quadrant(const double *L, const double *Rm, int w, int lane) {
  const int qr = w >> 1, qc = w & 1, li = lane & 15, lk = lane >> 4;
  doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int st = 0; st < kSub / 4; ++st) {
    const int k = 4 * st + lk;
    const double av = TRANS_L ? L[k * kSubLd + 16 * qr + li] : L[(16 * qr + li) * kSubLd + k];
    const double bv = Rm[k * kSubLd + 16 * qc + li];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
  return acc;
}

// Rotate M (pair blocks) and V (row tiles x pair columns) in place:
// M[S_p, S_q] <- R_p^T M[S_p, S_q] R_q, V[:, S_q] <- V[:, S_q] R_q.  Each
// workgroup reads its whole block before writing it back.
__global__ __launch_bounds__(256) void bj_update_kernel(double *__restrict__ M, double *__restrict__ V,
                                                        int64_t lp, int nb, int step,
                                                        const double *__restrict__ R) {
  __shared__ double blk[kSub * kSubLd];
  __shared__ double tmp[kSub * kSubLd];
  __shared__ double rq[kSub * kSubLd];
  __shared__ double rp[kSub * kSubLd];
  const int npairs = nb / 2;
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int qr = w >> 1, qc = w & 1, li = lane & 15, lk = lane >> 4;
  const int64_t nm = (int64_t)npairs * npairs;
  const int64_t id = blockIdx.x;
  const bool is_m = id < nm;
  int p, q;
  int64_t rowtile = 0;
  if (is_m) { p = (int)(id / npairs); q = (int)(id % npairs); }
  else { const int64_t k = id - nm; rowtile = k / npairs; q = (int)(k % npairs); p = -1; }
  const int qi = rr_player(q, step, nb), qj = rr_player(nb - 1 - q, step, nb);
  for (int e = tid; e < kSub * kSub; e += 256) {
    rq[(e / kSub) * kSubLd + e % kSub] = R[(int64_t)q * kSub * kSub + e];
  }
  if (is_m) {
    const int pi = rr_player(p, step, nb), pj = rr_player(nb - 1 - p, step, nb);
    for (int e = tid; e < kSub * kSub; e += 256) {
      const int u = e / kSub, x = e % kSub;
      rp[u * kSubLd + x] = R[(int64_t)p * kSub * kSub + e];
      blk[u * kSubLd + x] = M[(int64_t)sub_index(u, pi, pj) * lp + sub_index(x, qi, qj)];
    }
    __syncthreads();
    const doublex4 t = mm32_quadrant<false>(blk, rq, w, lane);      // blk R_q
#pragma unroll
    for (int v = 0; v < 4; ++v) tmp[(16 * qr + 4 * v + lk) * kSubLd + 16 * qc + li] = t[v];
    __syncthreads();
    const doublex4 o = mm32_quadrant<true>(rp, tmp, w, lane);       // R_p^T (blk R_q)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      M[(int64_t)sub_index(16 * qr + 4 * v + lk, pi, pj) * lp + sub_index(16 * qc + li, qi, qj)] = o[v];
  } else {
    const int64_t r0 = rowtile * kSub;
    for (int e = tid; e < kSub * kSub; e += 256) {
      const int u = e / kSub, x = e % kSub;
      blk[u * kSubLd + x] = V[(r0 + u) * lp + sub_index(x, qi, qj)];
    }
    __syncthreads();
    const doublex4 o = mm32_quadrant<false>(blk, rq, w, lane);      // V_tile R_q
#pragma unroll
    for (int v = 0; v < 4; ++v) V[(r0 + 16 * qr + 4 * v + lk) * lp + sub_index(16 * qc + li, qi, qj)] = o[v];
  }
}

// floor = abs_factor * max |diag| (one workgroup over the diagonal).
__global__ __launch_bounds__(256) void bj_floor_kernel(const double *__restrict__ M, int64_t lp,
                                                       double abs_factor, int *__restrict__ count,
                                                       double *__restrict__ floor_abs) {
  __shared__ double mx[256];
  const int tid = threadIdx.x;
  double m = 0.0;
  for (int64_t i = tid; i < lp; i += 256) m = fmax(m, fabs(M[i * lp + i]));
  mx[tid] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) mx[tid] = fmax(mx[tid], mx[tid + s]);
    __syncthreads();
  }
  if (tid == 0) { floor_abs[0] = mx[0] * abs_factor; count[0] = 0; }
}

// Count the off-diagonal pairs that are not negligible (one row per thread
// block row; integer atomics, so the count is exact).
__global__ __launch_bounds__(256) void bj_check_kernel(const double *__restrict__ M, int64_t lp,
                                                       int *__restrict__ count,
                                                       const double *__restrict__ floor_abs,
                                                       double rel) {
  const int64_t i = blockIdx.x;
  const double fl = floor_abs[0];
  const double aii = M[i * lp + i];
  int c = 0;
  for (int64_t j = i + 1 + threadIdx.x; j < lp; j += 256)
    if (!negligible(M[i * lp + j], aii, M[j * lp + j], fl, rel)) ++c;
  if (c) atomicAdd(count, c);
}

__global__ void bj_init_kernel(const double *__restrict__ K, int64_t l, int64_t lp,
                               double *__restrict__ M, double *__restrict__ V) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= lp * lp) return;
  const int64_t i = e / lp, j = e % lp;
  M[e] = (i < l && j < l) ? K[i * l + j] : 0.0;
  V[e] = 0.0;
}

// Preconditioning: diagonalise every 64 x 64 diagonal block M[I, I] (the
// method's blocks make K nearly block-diagonal) and store its eigenvectors as
// the diagonal block V[I, I] of the starting basis.
constexpr int kPre = 64;
constexpr int kPreThreads = 1024;
__global__ __launch_bounds__(kPreThreads) void bj_pre_eig_kernel(const double *__restrict__ M, int64_t lp,
                                                         double *__restrict__ V, double rel) {
  __shared__ double a[kPre * kSmallLd];
  __shared__ double v[kPre * kSmallLd];
  __shared__ double fl;
  const int tid = threadIdx.x;
  const int64_t o = (int64_t)blockIdx.x * kPre;
  for (int e = tid; e < kPre * kPre; e += kPreThreads) {
    const int i = e / kPre, j = e % kPre;
    a[i * kSmallLd + j] = M[(o + i) * lp + o + j];
    v[i * kSmallLd + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < kPre; ++i) mx = fmax(mx, fabs(a[i * kSmallLd + i]));
    fl = mx * kJacobiAbs;
  }
  __syncthreads();
  jacobi_lds<kPre, kSmallLd, kPreThreads>(a, v, fl, kPreSweeps, rel);
  __syncthreads();
  for (int e = tid; e < kPre * kPre; e += kPreThreads) {
    const int i = e / kPre, j = e % kPre;
    V[(o + i) * lp + o + j] = v[i * kSmallLd + j];
  }
}

// M[I, J] <- W_I^T M[I, J] W_J with W_I = V[I, I] (64 x 64 blocks, in place:
// each workgroup reads and writes only its own block).
__global__ __launch_bounds__(256) void bj_pre_rotate_kernel(double *__restrict__ M,
                                                            const double *__restrict__ V, int64_t lp) {
  __shared__ double blk[kPre * kSmallLd];
  __shared__ double w[kPre * kSmallLd];
  const int tid = threadIdx.x;
  const int64_t oi = (int64_t)blockIdx.x * kPre, oj = (int64_t)blockIdx.y * kPre;
  // tmp = M_IJ W_J  (into blk after the first pass)
  for (int e = tid; e < kPre * kPre; e += 256) {
    const int i = e / kPre, j = e % kPre;
    blk[i * kSmallLd + j] = M[(oi + i) * lp + oj + j];
    w[i * kSmallLd + j] = V[(oj + i) * lp + oj + j];
  }
  __syncthreads();
  double t[16];
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q, i = e / kPre, j = e % kPre;
    double s = 0.0;
    for (int k = 0; k < kPre; ++k) s = fma(blk[i * kSmallLd + k], w[k * kSmallLd + j], s);
    t[q] = s;
  }
  __syncthreads();
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q, i = e / kPre, j = e % kPre;
    blk[i * kSmallLd + j] = t[q];
    w[i * kSmallLd + j] = V[(oi + i) * lp + oi + j];
  }
  __syncthreads();
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q, i = e / kPre, j = e % kPre;
    double s = 0.0;
    for (int k = 0; k < kPre; ++k) s = fma(w[k * kSmallLd + i], blk[k * kSmallLd + j], s);
    M[(oi + i) * lp + oj + j] = s;
  }
}

__global__ void bj_rank_kernel(const double *__restrict__ M, int64_t l, int64_t lp,
                               int *__restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const double wi = M[i * lp + i];
  int64_t rank = 0;
  for (int64_t j = 0; j < l; ++j) {
    const double wj = M[j * lp + j];
    rank += (wj > wi) || (wj == wi && j < i);
  }
  perm[rank] = (int)i;
}

__global__ void bj_gather_kernel(const double *__restrict__ M, const double *__restrict__ V,
                                 int64_t l, int64_t lp, const int *__restrict__ perm,
                                 double *__restrict__ w, double *__restrict__ Vout) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= l * l) return;
  const int64_t r = e / l, k = e % l;
  const int src = perm[k];
  Vout[e] = V[r * lp + src];
  if (r == 0) w[k] = M[(int64_t)src * lp + src];
}

static int64_t padded(int64_t l) { return (l + kPre - 1) / kPre * kPre; }

size_t eig_workspace_bytes(int64_t l) {
  const int64_t lp = padded(l);
  const int64_t nb = lp / kBlk;
  size_t bytes = 0;
  bytes += (size_t)lp * lp * 8 * 2;                 // M, V
  bytes += (size_t)(nb / 2) * kSub * kSub * 8;      // rotations
  bytes += (size_t)lp * 4 + 64;                     // perm, counters
  bytes += 256;
  return bytes;
}

int eig_sym(const double *K, int64_t l, double *w, double *Vout, void *work, double rel,
            hipStream_t st) {
  if (!(rel > 0.0)) rel = kJacobiRel;
  if (l <= 64) {
    launch_eig_small(K, (int)l, (int)l, w, Vout, (int)l, st);
    return 1;
  }
  const int64_t lp = padded(l);
  const int nb = (int)(lp / kBlk);
  const int npairs = nb / 2;
  char *p = static_cast<char *>(work);
  double *M = reinterpret_cast<double *>(p); p += (size_t)lp * lp * 8;
  double *V = reinterpret_cast<double *>(p); p += (size_t)lp * lp * 8;
  double *R = reinterpret_cast<double *>(p); p += (size_t)npairs * kSub * kSub * 8;
  int *perm = reinterpret_cast<int *>(p); p += (size_t)lp * 4;
  p = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(p) + 63) & ~uintptr_t(63));
  int *count = reinterpret_cast<int *>(p);
  double *floor_abs = reinterpret_cast<double *>(p + 8);

  const int64_t tot = lp * lp;
  // the rotations leave FP64 rounding in every entry that grows with the
  // order (measured: sweeps stall below about 4e-13 max |a_ii| at l = 1000
  // and 2e-12 at l = 2000); the floor follows l^2 u64 / 128 above 1e-13 so
  // that the sweeps stop at that level instead of running to the cap
  const double abs_factor =
      std::fmax(kJacobiAbs, (double)lp * (double)lp * 1.1102230246251565e-16 / 128.0);
  hipLaunchKernelGGL(bj_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, K, l, lp, M, V);
  const int npre = (int)(lp / kPre);
  hipLaunchKernelGGL(bj_pre_eig_kernel, dim3(npre), dim3(kPreThreads), 0, st, M, lp, V, rel);
  hipLaunchKernelGGL(bj_pre_rotate_kernel, dim3(npre, npre), dim3(256), 0, st, M, V, lp);
  int sweeps = 0;
  const int max_sweeps = 40;
  for (; sweeps < max_sweeps; ++sweeps) {
    hipLaunchKernelGGL(bj_floor_kernel, dim3(1), dim3(256), 0, st, M, lp, abs_factor, count, floor_abs);
    hipLaunchKernelGGL(bj_check_kernel, dim3((unsigned)lp), dim3(256), 0, st, M, lp, count, floor_abs,
                       rel);
    int h_count = 0;
    hipMemcpyAsync(&h_count, count, sizeof(int), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    if (h_count == 0) break;
    for (int step = 0; step < nb - 1; ++step) {
      hipLaunchKernelGGL(bj_pair_kernel, dim3(npairs), dim3(kPairThreads), 0, st, M, lp, nb, step, R, floor_abs,
                         rel);
      const int64_t nwg = (int64_t)npairs * npairs + (lp / kSub) * npairs;
      hipLaunchKernelGGL(bj_update_kernel, dim3((unsigned)nwg), dim3(256), 0, st, M, V, lp, nb, step, R);
    }
  }
  hipLaunchKernelGGL(bj_rank_kernel, dim3((unsigned)((l + 255) / 256)), dim3(256), 0, st, M, l, lp, perm);
  hipLaunchKernelGGL(bj_gather_kernel, dim3((unsigned)((l * l + 255) / 256)), dim3(256), 0, st, M, V,
                     l, lp, perm, w, Vout);
  return sweeps;
}

}  // namespace farpca_int
