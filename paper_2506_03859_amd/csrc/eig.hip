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
// output block depends only on the same input block: one workgroup per block,
// M into a second buffer (V in place), in the same launch as the next round's
// pair subproblems.  Sweeps repeat until every off-diagonal
// entry is negligible relative to its diagonal pair.  Padding rows/columns are
// exactly zero and never couple (their rotations are the identity).
#include <cmath>
#include <cstring>
#include <utility>

#include "internal.h"

namespace farpca_int {

// A pair (p, q) is left alone when |a_pq| <= rel sqrt(|a_pp a_qq|) (the
// relative test that keeps Jacobi's small eigenvalues accurate; rel = 1e-14
// unless the caller asks for less) or when |a_pq| <= 4e-15 max_i |a_ii|, just
// above the FP64 rounding the block updates leave in every entry (measured up
// to about 1e-15 max |a_ii| at l = 2000), below which no rotation can go.  The
// floor must stay near that level: the method's Grams span ten and more orders
// of magnitude (a rank-100 signal over noise: 8e8 down to 0.15), and
// V = C^T U~ S^-1 inherits a_pq / (s_p s_q) as its loss of orthogonality (a
// floor of 1e-13 max |a_ii| left the noise directions' V orthonormal only to
// 4e-4).
constexpr double kJacobiRel = 1e-14;
constexpr double kJacobiTiny = 4e-15;
// The block updates leave FP64 rounding in every entry, so the tests above
// may never be met by some entries: once two sweeps in a row halve neither the
// largest ratio |a_pq| / sqrt(|a_pp a_qq|) nor the largest |a_pq| among the
// entries that fail them (against their best values so far), and either is
// down at the rounding level (ratio below kStallRel, or |a_pq| below kStallAbs
// max |a_ii|), the sweeps have stalled and stop (counted as converged).
constexpr double kStallRel = 1e-11;
constexpr double kStallAbs = 1e-12;
constexpr int kInnerMaxSweeps = 30;   // a small matrix solved on its own
// Inside the block method a diagonal-block pre-rotation and a pair subproblem
// need not be converged: each is one step of the outer iteration, whose own
// test decides convergence.  (One inner sweep per pair costs about one more
// outer sweep than solving every pair exactly, at a small fraction of the work.)
constexpr int kPreSweeps = 2;
constexpr int kPairSweeps = 1;

__device__ __forceinline__ bool negligible(double apq, double app, double aqq, double floor_abs,
                                           double rel) {
  // |a_pq| <= rel sqrt(|a_pp a_qq|), compared in squares (no square root)
  const double x = fabs(apq);
  return x == 0.0 || x <= floor_abs || x * x <= rel * rel * fabs(app * aqq);
}

__device__ __forceinline__ int rr_player(int pos, int step, int n) {
  // circle method: position 0 fixed, the others rotate
  return pos == 0 ? 0 : ((pos - 1 + step) % (n - 1)) + 1;
}

// The player after x in the next step of the tournament (x in 0 .. S - 1):
// 0 stays, S - 1 wraps to 1, the others add one.
template <int S>
__device__ __forceinline__ int rr_next(int x) {
  const int y = x + 1;
  return (y - (y / S) * (S - 1)) * min(x, 1);
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

// Cyclic Jacobi on an S x S symmetric matrix (LDS, stride LD) accumulating
// the rotations into v (LDS, stride LD, holds the starting orthogonal matrix).
// A step rotates the S / 2 disjoint pairs (p_i, q_i) of a round-robin
// tournament.  The matrix is double-buffered: a step reads `cur` and writes
// `nxt`, and every thread computes the rotations it applies from `cur` itself
// (the same inputs and instructions in every thread, so all copies of a
// rotation are bitwise equal), which leaves one barrier per step.  Thread t
// owns the 2 x 2 blocks (pairs ia, ib) with ib = t mod S/2 and the rows of v
// congruent to t div S/2; an identity rotation is applied like any other
// (c = 1, s = 0 copy exactly).  A step issues all of its LDS reads first and
// computes its rotations without branches, so that it costs one LDS round
// trip and one rotation's latency (the pairs' players advance by one
// tournament step in registers).  Returns the buffer holding the result.
// *converged (if given, thread 0's copy is enough) tells whether a sweep ended
// without a rotation before max_sweeps ran out.
template <int S, int LD, int NT>
__device__ double *jacobi_lds(double *a, double *a2, double *v, double floor_abs, int max_sweeps,
                              double rel, bool *converged = nullptr) {
  constexpr int H = S / 2;
  constexpr int TR = NT / H;        // threads per pair index ib
  static_assert(NT % H == 0 && H % TR == 0 && S % TR == 0, "thread layout");
  constexpr int BPT = H / TR;       // 2 x 2 blocks of the matrix per thread
  constexpr int RPT = S / TR;       // rows of v per thread
  __shared__ int rot_flag[2];
  const int tid = threadIdx.x;
  const int ib = tid % H, i0 = tid / H;
  if (tid == 0) { rot_flag[0] = 0; rot_flag[1] = 0; }
  __syncthreads();
  // players of the thread's pairs (slot 0: pair ib; slots 1..: the pairs ia
  // of its blocks), advanced by one tournament step at a time
  int pr[BPT + 1], qr[BPT + 1];
#pragma unroll
  for (int k = 0; k <= BPT; ++k) {
    const int idx = k == 0 ? ib : i0 + (k - 1) * TR;
    pr[k] = rr_player(idx, 0, S);
    qr[k] = rr_player(S - 1 - idx, 0, S);
  }
  double *cur = a, *nxt = a2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    for (int step = 0; step < S - 1; ++step) {
      // the flag of the next sweep was last read before this sweep's first barrier
      if (step == 1 && tid == 0) rot_flag[(sweep + 1) & 1] = 0;
      const int pb = pr[0], qb = qr[0];
      // every LDS read of the step first (one round trip): the three entries
      // of each rotation, the thread's 2 x 2 blocks and its rows of v
      double app[BPT + 1], aqq[BPT + 1], apq[BPT + 1];
#pragma unroll
      for (int k = 0; k <= BPT; ++k) {
        app[k] = cur[pr[k] * LD + pr[k]];
        aqq[k] = cur[qr[k] * LD + qr[k]];
        apq[k] = cur[pr[k] * LD + qr[k]];
      }
      double x[BPT][4];
#pragma unroll
      for (int k = 1; k <= BPT; ++k) {
        x[k - 1][0] = cur[pr[k] * LD + pb];
        x[k - 1][1] = cur[pr[k] * LD + qb];
        x[k - 1][2] = cur[qr[k] * LD + pb];
        x[k - 1][3] = cur[qr[k] * LD + qb];
      }
      double vp[RPT], vq[RPT];
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = i0 + k * TR;
        vp[k] = v[r * LD + pb];
        vq[k] = v[r * LD + qb];
      }
      // the rotations, without branches (a negligible pair takes c = 1,
      // s = 0; the values computed for it are discarded)
      double cr[BPT + 1], sr[BPT + 1];
      bool rotated = false;
#pragma unroll
      for (int k = 0; k <= BPT; ++k) {
        double c, s;
        jacobi_rotation(app[k], aqq[k], apq[k], c, s);
        const bool neg = negligible(apq[k], app[k], aqq[k], floor_abs, rel);
        cr[k] = neg ? 1.0 : c;
        sr[k] = neg ? 0.0 : s;
        rotated |= !neg;
      }
      const double cb = cr[0], sb = sr[0];
#pragma unroll
      for (int k = 1; k <= BPT; ++k) {
        const double ca = cr[k], sa = sr[k];
        const int pa = pr[k], qa = qr[k];
        const double x11 = x[k - 1][0], x12 = x[k - 1][1], x21 = x[k - 1][2], x22 = x[k - 1][3];
        const double y11 = ca * x11 - sa * x21, y12 = ca * x12 - sa * x22;
        const double y21 = sa * x11 + ca * x21, y22 = sa * x12 + ca * x22;
        nxt[pa * LD + pb] = cb * y11 - sb * y12;
        nxt[pa * LD + qb] = sb * y11 + cb * y12;
        nxt[qa * LD + pb] = cb * y21 - sb * y22;
        nxt[qa * LD + qb] = sb * y21 + cb * y22;
      }
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = i0 + k * TR;
        v[r * LD + pb] = cb * vp[k] - sb * vq[k];
        v[r * LD + qb] = sb * vp[k] + cb * vq[k];
      }
      if (rotated) rot_flag[sweep & 1] = 1;
      // next step's players: player 0 stays, the others advance cyclically
      // through 1 .. S - 1 (in arithmetic: no divergent branches)
#pragma unroll
      for (int k = 0; k <= BPT; ++k) {
        pr[k] = rr_next<S>(pr[k]);
        qr[k] = rr_next<S>(qr[k]);
      }
      __syncthreads();
      double *t = cur; cur = nxt; nxt = t;
    }
    if (!rot_flag[sweep & 1]) {
      if (converged) *converged = true;
      return cur;
    }
  }
  if (converged) *converged = false;
  return cur;
}

constexpr int kSmallLd = 65;

// conv (may be null): set to 1 if the sweeps converged, 0 if they hit the cap.
__global__ __launch_bounds__(256) void eig_small_kernel(const double *__restrict__ K, int s, int ldk,
                                                        double *__restrict__ w, double *__restrict__ V,
                                                        int ldv, int *__restrict__ conv) {
  __shared__ double a0[64 * kSmallLd];
  __shared__ double a1[64 * kSmallLd];
  __shared__ double v[64 * kSmallLd];
  __shared__ double fl;
  __shared__ int perm[64];
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e / 64, j = e % 64;
    a0[i * kSmallLd + j] = (i < s && j < s) ? K[i * ldk + j] : 0.0;
    v[i * kSmallLd + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < s; ++i) mx = fmax(mx, fabs(a0[i * kSmallLd + i]));
    fl = mx * kJacobiTiny;
  }
  __syncthreads();
  bool ok = false;
  const double *a = jacobi_lds<64, kSmallLd, 256>(a0, a1, v, fl, kInnerMaxSweeps, kJacobiRel, &ok);
  if (conv && tid == 0) conv[0] = ok ? 1 : 0;
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
                      hipStream_t st, int *conv) {
  hipLaunchKernelGGL(eig_small_kernel, dim3(1), dim3(256), 0, st, K, s, ldk, w, Vout, ldv, conv);
}

// ------------------------------------------------------------- block Jacobi
constexpr int kBlk = 16;           // block width
constexpr int kSub = 2 * kBlk;     // subproblem size
constexpr int kSubLd = kSub + 1;
constexpr int kPairThreads = 256;

__device__ __forceinline__ int sub_index(int u, int bi, int bj) {
  return u < kBlk ? bi * kBlk + u : bj * kBlk + (u - kBlk);
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

// The pair index and half (0: first block, 1: second) of block x at
// tournament step `step`: the inverse of rr_player.
__device__ __forceinline__ void rr_slot(int x, int step, int nb, int &pair, int &half) {
  const int pos = x == 0 ? 0 : ((x - 1 - step) % (nb - 1) + (nb - 1)) % (nb - 1) + 1;
  pair = pos < nb / 2 ? pos : nb - 1 - pos;
  half = pos < nb / 2 ? 0 : 1;
}

// One Jacobi round is one launch: its first npairs workgroups solve the pair
// subproblems of tournament step `step` (one sweep of M[S, S] in LDS, S =
// block(bi) U block(bj); rotations to Rcur, fcur[pair] = 0 when no entry
// needed one, R = I exactly), the others apply the rotations of step - 1
// (Rprev, fprev) to the whole matrix:
// M[S_p, S_q] <- R_p^T M[S_p, S_q] R_q (from Msrc into Mdst; a block whose
// rotations are both the identity is copied), V[:, S_q] <- V[:, S_q] R_q (in
// place, each row tile by one workgroup).  The pair workgroups do not wait for
// that update: they form the four 16 x 16 blocks of their subproblem from
// Msrc and Rprev themselves, with the products, operands and order the update
// uses for those blocks, so they hold bitwise the values it writes.  The first
// round of a sweep reads its subproblems straight from Msrc; after the last,
// an update-only launch (no pair workgroups) applies its rotations.
constexpr int kRoundLds = 4 * kSub * kSubLd + 4 * kSub * 17;   // doubles

__device__ void pair_role(double *sh, const double *__restrict__ Msrc, int64_t lp, int nb, int step,
                          const double *__restrict__ Rprev, const int *__restrict__ fprev,
                          double *__restrict__ Rcur, int *__restrict__ fcur,
                          const double *__restrict__ floor_abs, double rel, int pair) {
  double *a = sh, *a2 = sh + kSub * kSubLd, *v = sh + 2 * kSub * kSubLd;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, li = lane & 15, lk = lane >> 4;
  const int bi = rr_player(pair, step, nb), bj = rr_player(nb - 1 - pair, step, nb);
  if (step == 0) {
    for (int e = tid; e < kSub * kSub; e += kPairThreads) {
      const int u = e / kSub, x = e % kSub;
      a[u * kSubLd + x] = Msrc[(int64_t)sub_index(u, bi, bj) * lp + sub_index(x, bi, bj)];
    }
  } else {
    // wave w: block (X, Y) = (w / 2, w % 2) of the subproblem, rows of block
    // x = X ? bj : bi, columns of block y = Y ? bj : bi
    const int X = w >> 1, Y = w & 1;
    const int x = X ? bj : bi, y = Y ? bj : bi;
    int px, hx, py, hy;
    rr_slot(x, step - 1, nb, px, hx);
    rr_slot(y, step - 1, nb, py, hy);
    if (fprev[px] == 0 && fprev[py] == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = 4 * t + lk;
        a[(16 * X + r) * kSubLd + 16 * Y + li] = Msrc[(int64_t)(16 * x + r) * lp + 16 * y + li];
      }
    } else {
      const int pi = rr_player(px, step - 1, nb), pj = rr_player(nb - 1 - px, step - 1, nb);
      const int qi = rr_player(py, step - 1, nb), qj = rr_player(nb - 1 - py, step - 1, nb);
      const double *Rp = Rprev + (int64_t)px * kSub * kSub;
      const double *Rq = Rprev + (int64_t)py * kSub * kSub;
      // columns 16 hy .. of T = M[S_px, S_py] R_py (the update's quadrants
      // (0, hy) and (1, hy)), then quadrant (hx, hy) of R_px^T T
      double *tw = sh + 3 * kSub * kSubLd + w * kSub * 17;
#pragma unroll
      for (int qr = 0; qr < 2; ++qr) {
        doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int st = 0; st < kSub / 4; ++st) {
          const int k = 4 * st + lk;
          const double av = Msrc[(int64_t)sub_index(16 * qr + li, pi, pj) * lp + sub_index(k, qi, qj)];
          const double bv = Rq[k * kSub + 16 * hy + li];
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) tw[(16 * qr + 4 * t + lk) * 17 + li] = acc[t];
      }
      // the wave reads back only what it wrote (a wave's LDS accesses run in order)
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      doublex4 o = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < kSub / 4; ++st) {
        const int k = 4 * st + lk;
        o = __builtin_amdgcn_mfma_f64_16x16x4f64(Rp[k * kSub + 16 * hx + li], tw[k * 17 + li], o, 0, 0, 0);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) a[(16 * X + 4 * t + lk) * kSubLd + 16 * Y + li] = o[t];
    }
  }
  for (int e = tid; e < kSub * kSub; e += kPairThreads) {
    const int u = e / kSub, x = e % kSub;
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
  if (any_big) jacobi_lds<kSub, kSubLd, kPairThreads>(a, a2, v, fl, kPairSweeps, rel);   // else R = I
  __syncthreads();
  double *Rw = Rcur + (int64_t)pair * kSub * kSub;
  for (int e = tid; e < kSub * kSub; e += kPairThreads) Rw[e] = v[(e / kSub) * kSubLd + (e % kSub)];
  if (tid == 0) fcur[pair] = any_big ? 1 : 0;
}

__device__ void update_role(double *sh, const double *__restrict__ Msrc, double *__restrict__ Mdst,
                            double *__restrict__ V, int64_t lp, int nb, int step,
                            const double *__restrict__ R, const int *__restrict__ rflag, int64_t id) {
  double *blk = sh, *tmp = sh + kSub * kSubLd, *rq = sh + 2 * kSub * kSubLd, *rp = sh + 3 * kSub * kSubLd;
  const int npairs = nb / 2;
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  const int qr = w >> 1, qc = w & 1, li = lane & 15, lk = lane >> 4;
  const int64_t nm = (int64_t)npairs * npairs;
  const bool is_m = id < nm;
  int p, q;
  int64_t rowtile = 0;
  if (is_m) { p = (int)(id / npairs); q = (int)(id % npairs); }
  else { const int64_t k = id - nm; rowtile = k / npairs; q = (int)(k % npairs); p = -1; }
  const int qi = rr_player(q, step, nb), qj = rr_player(nb - 1 - q, step, nb);
  if (rflag[q] == 0 && (!is_m || rflag[p] == 0)) {              // uniform: the whole workgroup
    if (is_m) {
      const int pi = rr_player(p, step, nb), pj = rr_player(nb - 1 - p, step, nb);
      for (int e = tid; e < kSub * kSub; e += 256) {
        const int64_t o = (int64_t)sub_index(e / kSub, pi, pj) * lp + sub_index(e % kSub, qi, qj);
        Mdst[o] = Msrc[o];
      }
    }
    return;
  }
  for (int e = tid; e < kSub * kSub; e += 256) {
    rq[(e / kSub) * kSubLd + e % kSub] = R[(int64_t)q * kSub * kSub + e];
  }
  if (is_m) {
    const int pi = rr_player(p, step, nb), pj = rr_player(nb - 1 - p, step, nb);
    for (int e = tid; e < kSub * kSub; e += 256) {
      const int u = e / kSub, x = e % kSub;
      rp[u * kSubLd + x] = R[(int64_t)p * kSub * kSub + e];
      blk[u * kSubLd + x] = Msrc[(int64_t)sub_index(u, pi, pj) * lp + sub_index(x, qi, qj)];
    }
    __syncthreads();
    const doublex4 t = mm32_quadrant<false>(blk, rq, w, lane);      // blk R_q
#pragma unroll
    for (int v = 0; v < 4; ++v) tmp[(16 * qr + 4 * v + lk) * kSubLd + 16 * qc + li] = t[v];
    __syncthreads();
    const doublex4 o = mm32_quadrant<true>(rp, tmp, w, lane);       // R_p^T (blk R_q)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      Mdst[(int64_t)sub_index(16 * qr + 4 * v + lk, pi, pj) * lp + sub_index(16 * qc + li, qi, qj)] = o[v];
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

__global__ __launch_bounds__(kPairThreads) void bj_round_kernel(
    const double *__restrict__ Msrc, double *__restrict__ Mdst, double *__restrict__ V, int64_t lp,
    int nb, int step, const double *__restrict__ Rprev, const int *__restrict__ fprev,
    double *__restrict__ Rcur, int *__restrict__ fcur, const double *__restrict__ floor_abs,
    double rel, int npair_wgs) {
  static_assert(kPairThreads == 256, "four waves: one per subproblem block and output quadrant");
  __shared__ double sh[kRoundLds];
  if ((int)blockIdx.x < npair_wgs)
    pair_role(sh, Msrc, lp, nb, step, Rprev, fprev, Rcur, fcur, floor_abs, rel, (int)blockIdx.x);
  else
    update_role(sh, Msrc, Mdst, V, lp, nb, step - 1, Rprev, fprev, (int64_t)blockIdx.x - npair_wgs);
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
  if (tid == 0) {
    floor_abs[0] = mx[0] * abs_factor;
    floor_abs[1] = mx[0];
    count[0] = 0;
    reinterpret_cast<unsigned long long *>(floor_abs)[2] = 0ull;
    reinterpret_cast<unsigned long long *>(floor_abs)[3] = 0ull;
  }
}

// Count the off-diagonal pairs that are not negligible and find their largest
// ratio |a_pq| / sqrt(|a_pp a_qq|) (one row per workgroup; integer atomics, so
// both are exact: a non-negative double orders like its bit pattern).
// stat = floor_abs: [0] the absolute floor, [1] max |a_ii|, [2] bits of the
// largest ratio, [3] bits of the largest |a_pq| (both over the failing pairs).
__global__ __launch_bounds__(256) void bj_check_kernel(const double *__restrict__ M, int64_t lp,
                                                       int *__restrict__ count,
                                                       double *__restrict__ stat, double rel) {
  __shared__ double mx[256];
  const int64_t i = blockIdx.x;
  const double fl = stat[0];
  const double aii = M[i * lp + i];
  __shared__ double mxa[256];
  int c = 0;
  double m = 0.0, ma = 0.0;
  for (int64_t j = i + 1 + threadIdx.x; j < lp; j += 256) {
    const double x = M[i * lp + j], ajj = M[j * lp + j];
    if (!negligible(x, aii, ajj, fl, rel)) {
      ++c;
      // ratio to the pair's diagonal (infinite for a nonzero entry beside a
      // zero diagonal entry)
      const double d = sqrt(fabs(aii * ajj));
      m = fmax(m, d > 0.0 ? fabs(x) / d : __builtin_inf());
      ma = fmax(ma, fabs(x));
    }
  }
  if (c) atomicAdd(count, c);
  mx[threadIdx.x] = m;
  mxa[threadIdx.x] = ma;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + s]);
      mxa[threadIdx.x] = fmax(mxa[threadIdx.x], mxa[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && mx[0] > 0.0) {
    atomicMax(reinterpret_cast<unsigned long long *>(stat) + 2,
              (unsigned long long)__double_as_longlong(mx[0]));
    atomicMax(reinterpret_cast<unsigned long long *>(stat) + 3,
              (unsigned long long)__double_as_longlong(mxa[0]));
  }
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
  __shared__ double a2[kPre * kSmallLd];
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
    fl = mx * kJacobiTiny;
  }
  __syncthreads();
  jacobi_lds<kPre, kSmallLd, kPreThreads>(a, a2, v, fl, kPreSweeps, rel);
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
  bytes += (size_t)lp * lp * 8 * 3;                 // M (two buffers), V
  bytes += (size_t)(nb / 2) * kSub * kSub * 8 * 2;  // rotations of two rounds
  bytes += (size_t)lp * 4 + 64;                     // perm, counters
  bytes += (size_t)(nb / 2) * 4 * 2 + 64;           // per-pair rotation flags of two rounds
  bytes += 256;
  return bytes;
}

int eig_sym(const double *K, int64_t l, double *w, double *Vout, void *work, double rel,
            hipStream_t st, bool *converged) {
  if (!(rel > 0.0)) rel = kJacobiRel;
  if (l <= 64) {
    int *conv = reinterpret_cast<int *>(static_cast<char *>(work) + eig_workspace_bytes(l) - 64);
    launch_eig_small(K, (int)l, (int)l, w, Vout, (int)l, st, conv);
    int h_conv = 0;
    hipMemcpyAsync(&h_conv, conv, sizeof(int), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    if (converged) *converged = h_conv == 1;
    return 1;
  }
  const int64_t lp = padded(l);
  const int nb = (int)(lp / kBlk);
  const int npairs = nb / 2;
  char *p = static_cast<char *>(work);
  double *M = reinterpret_cast<double *>(p); p += (size_t)lp * lp * 8;
  double *M2 = reinterpret_cast<double *>(p); p += (size_t)lp * lp * 8;
  double *V = reinterpret_cast<double *>(p); p += (size_t)lp * lp * 8;
  double *Rb[2];
  Rb[0] = reinterpret_cast<double *>(p); p += (size_t)npairs * kSub * kSub * 8;
  Rb[1] = reinterpret_cast<double *>(p); p += (size_t)npairs * kSub * kSub * 8;
  int *perm = reinterpret_cast<int *>(p); p += (size_t)lp * 4;
  int *fb[2];
  fb[0] = reinterpret_cast<int *>(p); p += (size_t)npairs * 4;
  fb[1] = reinterpret_cast<int *>(p); p += (size_t)npairs * 4;
  p = reinterpret_cast<char *>((reinterpret_cast<uintptr_t>(p) + 63) & ~uintptr_t(63));
  int *count = reinterpret_cast<int *>(p);
  double *floor_abs = reinterpret_cast<double *>(p + 8);

  const int64_t tot = lp * lp;
  const double abs_factor = kJacobiTiny;
  hipLaunchKernelGGL(bj_init_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, K, l, lp, M, V);
  const int npre = (int)(lp / kPre);
  hipLaunchKernelGGL(bj_pre_eig_kernel, dim3(npre), dim3(kPreThreads), 0, st, M, lp, V, rel);
  hipLaunchKernelGGL(bj_pre_rotate_kernel, dim3(npre, npre), dim3(256), 0, st, M, V, lp);
  int sweeps = 0;
  bool conv = false;
  double best_ratio = 0.0, best_offa = 0.0;
  int flat_sweeps = 0;
  for (;;) {
    hipLaunchKernelGGL(bj_floor_kernel, dim3(1), dim3(256), 0, st, M, lp, abs_factor, count, floor_abs);
    hipLaunchKernelGGL(bj_check_kernel, dim3((unsigned)lp), dim3(256), 0, st, M, lp, count, floor_abs,
                       rel);
    // count (int, then padding), floor, max |a_ii|, largest ratio, largest |a_pq|
    double h_stat[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    hipMemcpyAsync(h_stat, count, sizeof(h_stat), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    int h_count = 0;
    std::memcpy(&h_count, &h_stat[0], sizeof(int));
    const double diag = h_stat[2], ratio = h_stat[3], offa = h_stat[4];
    if (h_count == 0) { conv = true; break; }
    // a sweep improves when it halves either measure's best value so far;
    // two sweeps in a row without improvement count as a stall
    const bool improved = sweeps == 0 || ratio < 0.5 * best_ratio || offa < 0.5 * best_offa;
    flat_sweeps = improved ? 0 : flat_sweeps + 1;
    if (sweeps == 0 || ratio < best_ratio) best_ratio = ratio;
    if (sweeps == 0 || offa < best_offa) best_offa = offa;
    if (flat_sweeps >= 2 && (ratio <= kStallRel || offa <= kStallAbs * diag)) { conv = true; break; }
    if (sweeps == kEigMaxSweeps) break;
    ++sweeps;
    // round 0: pair subproblems only; rounds 1 .. nb - 2: the previous
    // round's update and this round's pairs in one launch; then the last
    // round's update alone.  M moves between the two buffers with every update.
    const int64_t nwg = (int64_t)npairs * npairs + (lp / kSub) * npairs;
    for (int step = 0; step < nb; ++step) {
      const bool pairs = step < nb - 1, update = step > 0;
      const int64_t grid = (pairs ? npairs : 0) + (update ? nwg : 0);
      hipLaunchKernelGGL(bj_round_kernel, dim3((unsigned)grid), dim3(kPairThreads), 0, st, M, M2, V, lp, nb,
                         step, Rb[(step + 1) & 1], fb[(step + 1) & 1], Rb[step & 1], fb[step & 1], floor_abs,
                         rel, pairs ? npairs : 0);
      if (update) std::swap(M, M2);
    }
  }
  hipLaunchKernelGGL(bj_rank_kernel, dim3((unsigned)((l + 255) / 256)), dim3(256), 0, st, M, l, lp, perm);
  hipLaunchKernelGGL(bj_gather_kernel, dim3((unsigned)((l * l + 255) / 256)), dim3(256), 0, st, M, V,
                     l, lp, perm, w, Vout);
  if (converged) *converged = conv;
  return sweeps;
}

}  // namespace farpca_int
