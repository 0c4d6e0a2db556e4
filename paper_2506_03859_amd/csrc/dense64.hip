// FP64 work on the small dimensions of the method: b x b Gram matrices and
// their Cholesky factors (the orthonormalisation that replaces eigSVD, and the
// basis extension of the indicator step), the setup pass (||A||_F^2 and, for
// the standardized Bernoulli matrix, z = A (p 1_n)), and the indicator update
// E = ||A||_F^2 - sum_j ||C_j||_F^2 (the identity of Section 2.1).
// All reductions use a fixed partition and a fixed order: results are
// bitwise repeatable.
#include "internal.h"

namespace farpca_int {

typedef double doublex4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ------------------------------------------------------------------ Gram
// part[blk][i][j] = sum over the rows of block blk of X[k][i] X[k][j] (FP64;
// columns >= b read as zero), then G = sum of the partials in block order.
// Up to kGramParts workgroups, each over a contiguous row range in chunks of
// 128 rows staged in LDS (all of a chunk's loads in flight at once), products
// on the FP64 matrix cores.
constexpr int kGramParts = 256;
constexpr int kGramChunk = 128;   // rows staged per step: one step per workgroup up to 32768 rows

int gram_max_partials() { return kGramParts; }

__global__ __launch_bounds__(256) void gram_kernel(const float *__restrict__ X, int64_t ldx,
                                                   int64_t K, int b, int64_t rows_per_blk,
                                                   bool vec, double *__restrict__ part) {
  __shared__ float xs[kGramChunk][kMaxBlock + 1];
  const int t = threadIdx.x;
  // wave w forms the output blocks (w, 0 .. 3) (16 x 16 each) on the FP64
  // matrix cores, K = the chunk's rows: lane l supplies X^T (row l % 16,
  // k l / 16) and X (k l / 16, col l % 16); result element v of lane l is
  // (row 4 v + l / 16, col l % 16).  FP32 values enter exactly.
  const int w = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  doublex4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = doublex4{0.0, 0.0, 0.0, 0.0};
  const int64_t k_begin = (int64_t)blockIdx.x * rows_per_blk;
  int64_t k_end = k_begin + rows_per_blk;
  if (k_end > K) k_end = K;
  for (int64_t k0 = k_begin; k0 < k_end; k0 += kGramChunk) {
    const int nr = (int)((k_end - k0 < kGramChunk) ? k_end - k0 : kGramChunk);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kGramChunk * kMaxBlock / 4 / 256; ++q) {
      const int f = t + 256 * q;
      const int r = f >> 4, c4 = (f & 15) * 4;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (r < nr) {
        const float *p = X + (k0 + r) * ldx + c4;
        if (vec) v = *reinterpret_cast<const float4 *>(p);
        else v = make_float4(p[0], p[1], p[2], p[3]);
      }
      xs[r][c4 + 0] = (c4 + 0 < b) ? v.x : 0.0f;
      xs[r][c4 + 1] = (c4 + 1 < b) ? v.y : 0.0f;
      xs[r][c4 + 2] = (c4 + 2 < b) ? v.z : 0.0f;
      xs[r][c4 + 3] = (c4 + 3 < b) ? v.w : 0.0f;
    }
    __syncthreads();
    const int steps = (nr + 3) / 4;              // rows past nr are zero
    for (int st = 0; st < steps; ++st) {
      const int r = 4 * st + lk;
      const double av = (double)xs[r][16 * w + li];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, (double)xs[r][16 * c + li], acc[c], 0, 0, 0);
    }
  }
  double *o = part + (int64_t)blockIdx.x * kMaxBlock * kMaxBlock;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) o[(16 * w + 4 * v + lk) * kMaxBlock + 16 * c + li] = acc[c][v];
}

// G[e] = sum_q part[q][e] in a fixed order: workgroup g owns 16 entries; its
// 16 thread groups sum the partials q = grp, grp + 16, ... and the group sums
// are added in group order.
__global__ __launch_bounds__(256) void gram_reduce_kernel(const double *__restrict__ part, int nblk,
                                                          int b, double *__restrict__ G) {
  __shared__ double red[16][16];
  const int t = threadIdx.x;
  const int grp = t >> 4, o = t & 15;
  const int e = blockIdx.x * 16 + o;
  double s = 0.0;
  for (int q = grp; q < nblk; q += 16) s += part[(int64_t)q * kMaxBlock * kMaxBlock + e];
  red[grp][o] = s;
  __syncthreads();
  if (grp == 0) {
    double tot = 0.0;
#pragma unroll
    for (int g = 0; g < 16; ++g) tot += red[g][o];
    const int i = e / kMaxBlock, j = e % kMaxBlock;
    G[e] = (i < b && j < b) ? tot : 0.0;
  }
}

static int64_t gram_rows_per_blk(int64_t K) {
  int64_t rows = (K + kGramParts - 1) / kGramParts;
  if (rows < 16) rows = 16;
  return rows;
}

int gram_num_partials(int64_t K) {
  const int64_t rows = gram_rows_per_blk(K);
  return (int)((K + rows - 1) / rows);
}

void launch_gram(const float *X, int64_t ldx, int64_t K, int b, double *part, double *G,
                 hipStream_t st) {
  const int64_t rows = gram_rows_per_blk(K);
  const int nblk = K > 0 ? (int)((K + rows - 1) / rows) : 0;
  const bool vec = (ldx % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0);
  if (nblk > 0)
    hipLaunchKernelGGL(gram_kernel, dim3(nblk), dim3(256), 0, st, X, ldx, K, b, rows, vec, part);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(kMaxBlock * kMaxBlock / 16), dim3(256), 0, st, part,
                     nblk, b, G);
}

// ------------------------------------------------------- Cholesky factor
// G (kMaxBlock x kMaxBlock, FP64, valid b x b) = R^T R.  The output F holds R
// strictly above the diagonal and F_jj = 1 / R_jj on it (zero below): what
// the row-wise triangular solve X <- X R^{-1} needs.  A column whose pivot
// after elimination falls to drop_rel * (its own diagonal) or below is
// numerically dependent on the previous ones (for FP32 data the residual is
// rounding noise): it is dropped - its row of R is zero, so it eliminates
// nothing later, and F_jj = 0, so that output column is exactly zero.
// flags[0] |= 1 when a column is dropped.  (The method's Z^{-1} is read as
// the pseudo-inverse there.)
//
// One wave: lane j holds column j of the working matrix in registers; step k
// broadcasts the pivot and row k of R through LDS and updates the trailing
// columns.
constexpr int kInvLd = kMaxBlock + 1;      // LDS stride of the factor and its inverse

__device__ __forceinline__ double bcast_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

__global__ __launch_bounds__(64) void chol_kernel(const double *__restrict__ G, int b,
                                                  double drop_rel, double *__restrict__ F,
                                                  int *__restrict__ flags, double skip_tol,
                                                  int *__restrict__ apply) {
  __shared__ double rk[kMaxBlock];
  const int j = threadIdx.x;
  double c[kMaxBlock];
#pragma unroll
  for (int i = 0; i < kMaxBlock; ++i) c[i] = G[i * kMaxBlock + j];
  const double dg = G[j * kMaxBlock + j];
  if (skip_tol > 0.0) {
    // G of already orthonormal columns (a repeated pass): when every kept
    // column (nonzero diagonal) is orthonormal to skip_tol, R = I and the
    // solve is left out (apply[0] = 0)
    double dev = 0.0;
#pragma unroll
    for (int i = 0; i < kMaxBlock; ++i) {
      const bool kept = j < b && i < b && dg != 0.0 && G[i * kMaxBlock + i] != 0.0;
      const double e = kept ? fabs(c[i] - (i == j ? 1.0 : 0.0)) : 0.0;
      dev = (e > dev || e != e) ? e : dev;              // NaN counts as a deviation
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(dev, off);
      dev = (o > dev || o != o) ? o : dev;
    }
    const bool skip = dev <= skip_tol;                  // false for NaN
    if (j == 0) apply[0] = skip ? 0 : 1;
    if (skip) return;
  } else if (apply && j == 0) {
    apply[0] = 1;
  }
  // Right-looking factorization in panels of 16 pivots.  The working matrix
  // (upper triangle) lives in LDS.  Within a panel every lane j >= the
  // panel's first pivot keeps the panel's 16 rows of its column in registers
  // and takes the 16 pivot steps exactly as the unblocked algorithm does on
  // those rows (pivot, scaling, rank-1 update of the later panel rows).  The
  // rows below the panel are then updated in one step on the FP64 matrix
  // cores: A_ij -= sum over the panel's pivots k of R_ki R_kj (the
  // accumulator starts at A_ij).  R goes to Rl: R_kj above the diagonal,
  // F_kk = 1 / R_kk on it, rows of dropped pivots and columns >= b zero.
  __shared__ double Al[kMaxBlock * kInvLd];
  __shared__ double Rl[kMaxBlock * kInvLd];
  __shared__ double Ml[kMaxBlock * kInvLd];
  __shared__ double Tl[16 * 17];
#pragma unroll
  for (int i = 0; i < kMaxBlock; ++i) {
    Al[i * kInvLd + j] = c[i];
    Rl[i * kInvLd + j] = 0.0;
    Ml[i * kInvLd + j] = 0.0;
  }
  __syncthreads();
  const int li = j & 15, lk = j >> 4;
  bool any_drop = false;
  for (int p = 0; p < 4; ++p) {
    const int k0 = 16 * p;
    if (k0 >= b) break;
    double x[16];
#pragma unroll
    for (int il = 0; il < 16; ++il) x[il] = Al[(k0 + il) * kInvLd + j];
#pragma unroll
    for (int kl = 0; kl < 16; ++kl) {
      const int k = k0 + kl;
      if (k < b) {
        const double piv = bcast_f64(x[kl], k);
        const double dgk = bcast_f64(dg, k);
        double r = 0.0;                               // R[k][j] for j > k
        if (piv > drop_rel * dgk && piv > 0.0) {     // false for NaN too
          const double inv = rsqrt(piv);
          r = (j > k) ? x[kl] * inv : 0.0;
          x[kl] = (j == k) ? inv : ((j > k) ? r : x[kl]);
        } else {
          any_drop = true;
          x[kl] = (j >= k) ? 0.0 : x[kl];
        }
        rk[j] = r;
        __syncthreads();
#pragma unroll
        for (int il = kl + 1; il < 16; ++il) x[il] = fma(-rk[k0 + il], r, x[il]);
        __syncthreads();
      }
    }
#pragma unroll
    for (int il = 0; il < 16; ++il)
      Rl[(k0 + il) * kInvLd + j] = (j >= k0 + il && j < b && k0 + il < b) ? x[il] : 0.0;
    __syncthreads();
    for (int ti = p + 1; ti < 4; ++ti) {
      for (int tj = ti; tj < 4; ++tj) {
        doublex4 acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[v] = Al[(16 * ti + 4 * v + lk) * kInvLd + 16 * tj + li];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int kk = k0 + 4 * st + lk;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-Rl[kk * kInvLd + 16 * ti + li],
                                                     Rl[kk * kInvLd + 16 * tj + li], acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Al[(16 * ti + 4 * v + lk) * kInvLd + 16 * tj + li] = acc[v];
      }
    }
    __syncthreads();
  }
  if (any_drop && j == 0) atomicOr(flags, 1);
  // Rl: R[i][j] for i < j, F_jj = 1 / R_jj on the diagonal (0 for a dropped
  // column, whose row of R is zero too); columns >= b are zero.  The solve
  // y_c = F_cc (x_c - sum_{i<c} y_i R_ic) is linear in x: y = x M with M the
  // inverse of R (rows and columns of dropped pivots zero, since F_kk = 0
  // there).  M is formed here once, so that the row solve is a plain product.
  // diagonal 16 x 16 blocks by back substitution: lane j forms column j of
  // its block, M_jj = F_jj, M_ij = -F_ii sum_{i<k<=j} R_ik M_kj
  {
    const int blk = j >> 4, jl = j & 15, o = 16 * blk;
    double m[16];
#pragma unroll
    for (int il = 0; il < 16; ++il) m[il] = (il == jl) ? Rl[j * kInvLd + j] : 0.0;
#pragma unroll
    for (int il = 14; il >= 0; --il) {
      double acc = 0.0;
#pragma unroll
      for (int kl = il + 1; kl < 16; ++kl) acc = fma(Rl[(o + il) * kInvLd + o + kl], m[kl], acc);
      if (il < jl) m[il] = -Rl[(o + il) * kInvLd + o + il] * acc;
    }
#pragma unroll
    for (int il = 0; il < 16; ++il) Ml[(o + il) * kInvLd + j] = m[il];
  }
  __syncthreads();
  // off-diagonal blocks, nearest the diagonal first:
  // M_ab = -M_aa (sum_{a<c<=b} R_ac M_cb), as 16 x 16 products on the FP64
  // matrix cores (lane l: A (row l % 16, k l / 16), B (k l / 16, col l % 16),
  // result element v at (row 4 v + l / 16, col l % 16))
  for (int d = 1; d < 4; ++d) {
    for (int a = 0; a + d < 4; ++a) {
      const int bb = a + d;
      doublex4 t = {0.0, 0.0, 0.0, 0.0};
      for (int st = 0; st < 4 * d; ++st) {
        const int k = 16 * (a + 1) + 4 * st + lk;
        t = __builtin_amdgcn_mfma_f64_16x16x4f64(Rl[(16 * a + li) * kInvLd + k],
                                                 Ml[k * kInvLd + 16 * bb + li], t, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) Tl[(4 * v + lk) * 17 + li] = t[v];
      __syncthreads();
      doublex4 u = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int k = 4 * st + lk;
        u = __builtin_amdgcn_mfma_f64_16x16x4f64(Ml[(16 * a + li) * kInvLd + 16 * a + k],
                                                 Tl[k * 17 + li], u, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) Ml[(16 * a + 4 * v + lk) * kInvLd + 16 * bb + li] = -u[v];
      __syncthreads();
    }
  }
  // M stored by columns (lane j writes column j, contiguous)
#pragma unroll
  for (int i = 0; i < kMaxBlock; ++i) F[j * kMaxBlock + i] = Ml[i * kInvLd + j];
}

void launch_chol(const double *G, int b, double drop_rel, double *F, int *flags, double skip_tol,
                 int *apply, hipStream_t st) {
  hipLaunchKernelGGL(chol_kernel, dim3(1), dim3(64), 0, st, G, b, drop_rel, F, flags, skip_tol, apply);
}

// Y = X R^{-1} = X M (M the inverse formed by chol_kernel, stored by
// columns), FP64 products of the FP32 rows, each value rounded once to FP32.
// A workgroup (4 waves) per 64 rows: the row tile is read coalesced into LDS
// (row stride 65 floats) and M transposed into LDS (row stride 65 doubles);
// wave w forms rows 16 w .. 16 w + 15 of the product on the FP64 matrix cores
// (four 16 x 16 output blocks, K = 64) and writes them back into its own rows
// of the tile, which leaves coalesced.  Columns >= b are not written.  Y may
// alias X (a tile is read completely before any of it is written).
constexpr int kTrsmRows = 64;
__global__ __launch_bounds__(256) void trsm_rows_kernel(const float *__restrict__ X, int64_t ldx,
                                                        int64_t K, int b, const double *__restrict__ Fg,
                                                        float *__restrict__ Y, int64_t ldy, int vec,
                                                        const int *__restrict__ apply) {
  __shared__ double Ml[kMaxBlock * kInvLd];           // Ml[i][c] = M_ic
  __shared__ float xt[kTrsmRows * (kMaxBlock + 1)];
  if (apply && apply[0] == 0) return;                    // R = I: nothing to do (in place)
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * kTrsmRows;
  for (int e = t; e < kMaxBlock * kMaxBlock; e += 256)
    Ml[(e % kMaxBlock) * kInvLd + e / kMaxBlock] = Fg[e];
  // tile in: instruction q covers rows 4 q + t / 16, columns 4 (t % 16) .. + 3
#pragma unroll
  for (int q = t >> 4; q < kTrsmRows; q += 16) {
    const int row = q, c4 = 4 * (t & 15);
    const int64_t gr = r0 + row;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (gr < K) {
      const float *xr = X + gr * ldx + c4;
      if (vec) {
        const float4 u = *reinterpret_cast<const float4 *>(xr);
        v[0] = u.x; v[1] = u.y; v[2] = u.z; v[3] = u.w;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = (c4 + i < b) ? xr[i] : 0.f;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) xt[row * (kMaxBlock + 1) + c4 + i] = (c4 + i < b) ? v[i] : 0.f;
  }
  __syncthreads();
  const int w = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  doublex4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = doublex4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int st = 0; st < kMaxBlock / 4; ++st) {
    const int k = 4 * st + lk;
    const double av = (double)xt[(16 * w + li) * (kMaxBlock + 1) + k];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Ml[k * kInvLd + 16 * ct + li], acc[ct], 0, 0, 0);
  }
  // own rows only: no other wave reads them until the barrier
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      xt[(16 * w + 4 * v + lk) * (kMaxBlock + 1) + 16 * ct + li] = (float)acc[ct][v];
  __syncthreads();
#pragma unroll
  for (int q = t >> 4; q < kTrsmRows; q += 16) {
    const int row = q, c4 = 4 * (t & 15);
    const int64_t gr = r0 + row;
    if (gr >= K || c4 >= b) continue;
    float *yr = Y + gr * ldy + c4;
    const float *src = xt + row * (kMaxBlock + 1) + c4;
    if (vec && c4 + 4 <= b) {
      *reinterpret_cast<float4 *>(yr) = make_float4(src[0], src[1], src[2], src[3]);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (c4 + i < b) yr[i] = src[i];
    }
  }
}

void launch_trsm_rows(const float *X, int64_t ldx, int64_t K, int b, const double *F, float *Y,
                      int64_t ldy, const int *apply, hipStream_t st) {
  if (K <= 0) return;
  const int vec = (ldx % 4 == 0) && (ldy % 4 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                  ((reinterpret_cast<uintptr_t>(Y) & 15) == 0) && b == kMaxBlock;
  hipLaunchKernelGGL(trsm_rows_kernel, dim3((unsigned)((K + kTrsmRows - 1) / kTrsmRows)), dim3(256), 0,
                     st, X, ldx, K, b, F, Y, ldy, vec, apply);
}

// ------------------------------------------------------------ setup pass
// One wave per row at a time; each workgroup (4 waves) owns a fixed row range.
constexpr int kSetupWgs = 1024;

// Element loads: FP32, or BF16 bit patterns widened exactly.
__device__ __forceinline__ float elem(const float *p, int64_t c) { return p[c]; }
__device__ __forceinline__ float elem(const uint16_t *p, int64_t c) {
  return __uint_as_float((uint32_t)p[c] << 16);
}
__device__ __forceinline__ float4 elem4(const float *p, int64_t c4) {
  return reinterpret_cast<const float4 *>(p)[c4];
}
__device__ __forceinline__ float4 elem4(const uint16_t *p, int64_t c4) {
  const uint2 u = reinterpret_cast<const uint2 *>(p)[c4];
  return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xFFFF0000u),
                     __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xFFFF0000u));
}

template <typename T, bool VEC>
__global__ __launch_bounds__(256) void setup_kernel(const T *__restrict__ A, int64_t lda,
                                                    int64_t m, int64_t n, int64_t rows_per_wg,
                                                    double *__restrict__ part_sq,
                                                    double *__restrict__ rowsum,
                                                    int *__restrict__ flags) {
  __shared__ double wsum[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_wg;
  int64_t re = rb + rows_per_wg;
  if (re > m) re = m;
  double sq = 0.0;
  bool bad = false;
  for (int64_t row = rb + wave; row < re; row += 4) {
    const T *p = A + row * lda;
    double s = 0.0, q = 0.0;
    int64_t c0 = 0;
    if (VEC) {
      const int64_t n4 = n / 4;
      for (int64_t c = lane; c < n4; c += 64) {
        const float4 v = elem4(p, c);
        const double x0 = v.x, x1 = v.y, x2 = v.z, x3 = v.w;
        s += (x0 + x1) + (x2 + x3);
        q = fma(x0, x0, q); q = fma(x1, x1, q); q = fma(x2, x2, q); q = fma(x3, x3, q);
        bad |= !isfinite(v.x) || !isfinite(v.y) || !isfinite(v.z) || !isfinite(v.w);
      }
      c0 = n4 * 4;
    }
    for (int64_t c = c0 + lane; c < n; c += 64) {
      const float f = elem(p, c);
      const double x = f;
      s += x; q = fma(x, x, q);
      bad |= !isfinite(f);
    }
    s = wave_sum(s);
    q = wave_sum(q);
    if (lane == 0) rowsum[row] = s;
    sq += q;
  }
  if (bad) atomicOr(flags, 2);
  if (lane == 0) wsum[wave] = sq;
  __syncthreads();
  if (threadIdx.x == 0) part_sq[blockIdx.x] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

int setup_num_partials(int64_t m) {
  const int64_t rows = (m + kSetupWgs - 1) / kSetupWgs;
  return (int)((m + rows - 1) / rows);
}

template <typename T>
static void launch_setup_t(const T *A, int64_t lda, int64_t m, int64_t n, double *part_sq,
                           double *rowsum, int *flags, hipStream_t st) {
  const int64_t rows = (m + kSetupWgs - 1) / kSetupWgs;
  const int nwg = (int)((m + rows - 1) / rows);
  const bool vec = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & (4 * sizeof(T) - 1)) == 0);
  if (vec) hipLaunchKernelGGL((setup_kernel<T, true>), dim3(nwg), dim3(256), 0, st, A, lda, m, n,
                              rows, part_sq, rowsum, flags);
  else hipLaunchKernelGGL((setup_kernel<T, false>), dim3(nwg), dim3(256), 0, st, A, lda, m, n,
                          rows, part_sq, rowsum, flags);
}

void launch_setup(const void *A, bool bf16, int64_t lda, int64_t m, int64_t n, double *part_sq,
                  double *rowsum, int *flags, hipStream_t st) {
  if (bf16)
    launch_setup_t(static_cast<const uint16_t *>(A), lda, m, n, part_sq, rowsum, flags, st);
  else
    launch_setup_t(static_cast<const float *>(A), lda, m, n, part_sq, rowsum, flags, st);
}

// ------------------------------------------------------ fixed-order sums
__global__ __launch_bounds__(256) void sum_partials_kernel(const double *__restrict__ part, int count,
                                                           double *__restrict__ out, int mode,
                                                           double *__restrict__ hist, int64_t j) {
  __shared__ double ws[4];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int q = t; q < count; q += 256) s += part[q];
  s = wave_sum(s);
  if ((t & 63) == 0) ws[t >> 6] = s;
  __syncthreads();
  if (t == 0) {
    const double tot = ((ws[0] + ws[1]) + ws[2]) + ws[3];
    if (mode == 0) {
      out[0] = tot;
    } else {          // indicator: E -= tot, record history
      const double e = out[0] - tot;
      out[0] = e;
      if (hist) hist[j] = e;
    }
  }
}

void launch_sum_partials(const double *part, int count, double *out, hipStream_t st) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, st, part, count, out, 0,
                     (double *)nullptr, (int64_t)0);
}

void launch_indicator_update(const double *part, int count, double *E, double *E_hist, int64_t j,
                             hipStream_t st) {
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, st, part, count, E, 1, E_hist, j);
}

__global__ void scale_rowsum_kernel(const double *__restrict__ rowsum, int64_t m, double p,
                                    float *__restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) z[i] = (float)(p * rowsum[i]);
}

void launch_scale_rowsum(const double *rowsum, int64_t m, double p, float *z, hipStream_t st) {
  hipLaunchKernelGGL(scale_rowsum_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                     rowsum, m, p, z);
}

// ||X||_F^2 of a K x b block, one partial per workgroup (fixed partition).
constexpr int kSqWgs = 256;
__global__ __launch_bounds__(256) void sqnorm_kernel(const float *__restrict__ X, int64_t ldx,
                                                     int64_t K, int b, int64_t rows_per_wg,
                                                     double *__restrict__ part) {
  __shared__ double ws[4];
  const int t = threadIdx.x;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_wg;
  int64_t re = rb + rows_per_wg;
  if (re > K) re = K;
  double q = 0.0;
  const int c = t & 63;
  for (int64_t r = rb + (t >> 6); r < re; r += 4) {
    if (c < b) { const double x = X[r * ldx + c]; q = fma(x, x, q); }
  }
  q = wave_sum(q);
  if ((t & 63) == 0) ws[t >> 6] = q;
  __syncthreads();
  if (t == 0) part[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

int sqnorm_num_partials(int64_t K) {
  const int64_t rows = (K + kSqWgs - 1) / kSqWgs;
  return (int)((K + rows - 1) / rows);
}

void launch_sqnorm(const float *X, int64_t ldx, int64_t K, int b, double *part, hipStream_t st) {
  const int64_t rows = (K + kSqWgs - 1) / kSqWgs;
  const int nwg = (int)((K + rows - 1) / rows);
  hipLaunchKernelGGL(sqnorm_kernel, dim3(nwg), dim3(256), 0, st, X, ldx, K, b, rows, part);
}

// ------------------------------------------------------------ block helpers
__global__ void copy_block_kernel(const float *__restrict__ X, int64_t ldx, int64_t K, int b,
                                  float *__restrict__ D, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = idx / 64, c = idx % 64;
  if (r < K && c < b) D[r * ldd + c] = X[r * ldx + c];
}

void launch_copy_block(const float *X, int64_t ldx, int64_t K, int b, float *dst, int64_t ldd,
                       hipStream_t st) {
  const int64_t total = K * 64;
  hipLaunchKernelGGL(copy_block_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, X,
                     ldx, K, b, dst, ldd);
}

__global__ void axpy_block_kernel(float *__restrict__ X, int64_t ldx, const float *__restrict__ G,
                                  int64_t ldg, int64_t K, int b, const double *__restrict__ alpha) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = idx / 64, c = idx % 64;
  const float a = (float)alpha[0];
  if (r < K && c < b && a != 0.0f) X[r * ldx + c] -= a * G[r * ldg + c];
}

void launch_axpy_block(float *X, int64_t ldx, const float *G, int64_t ldg, int64_t K, int b,
                       const double *alpha_dev, hipStream_t st) {
  const int64_t total = K * 64;
  hipLaunchKernelGGL(axpy_block_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, X,
                     ldx, G, ldg, K, b, alpha_dev);
}

// Shift update of the power iteration (Algorithm 1 / 2): with s the smallest
// singular value of the block (sqrt of the smallest Gram eigenvalue),
// if alpha < s then alpha = (s + alpha) / 2.
__global__ void alpha_update_kernel(const double *__restrict__ w, int b, double *__restrict__ alpha) {
  double lmin = w[b - 1];           // eigenvalues in descending order
  if (lmin < 0.0) lmin = 0.0;
  const double s = sqrt(lmin);
  if (alpha[0] < s) alpha[0] = (s + alpha[0]) * 0.5;
}

void launch_alpha_update(const double *w, int b, double *alpha, hipStream_t st) {
  hipLaunchKernelGGL(alpha_update_kernel, dim3(1), dim3(1), 0, st, w, b, alpha);
}

}  // namespace farpca_int

namespace farpca_int {

constexpr int kGramRows = 32;   // rows staged per step of the big Gram

// ------------------------------------------------ final Gram K = X^T X (l x l)
// X is n x l FP32 (ldx).  Upper 64 x 64 tiles only; grid z splits the rows of
// X (partials part[z][lp][lp], reduced in a fixed order and mirrored).
__global__ __launch_bounds__(256) void gram_big_kernel(const float *__restrict__ X, int64_t ldx,
                                                       int64_t n, int64_t l, int64_t lp,
                                                       int64_t rows_per_split,
                                                       double *__restrict__ part) {
  const int ti_blk = blockIdx.x, tj_blk = blockIdx.y;
  if (tj_blk < ti_blk) return;
  __shared__ float xi_s[kGramRows][65];
  __shared__ float xj_s[kGramRows][65];
  const int t = threadIdx.x;
  // wave w forms rows 16 w .. 16 w + 15 of the 64 x 64 tile (four 16 x 16
  // blocks) on the FP64 matrix cores, K = the staged rows (FP32 values enter
  // exactly): lane l supplies X_i^T (row l % 16, k l / 16) and X_j (k l / 16,
  // col l % 16); result element v of lane l is (row 4 v + l / 16, col l % 16).
  const int w = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int64_t ci0 = (int64_t)ti_blk * 64, cj0 = (int64_t)tj_blk * 64;
  doublex4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = doublex4{0.0, 0.0, 0.0, 0.0};
  const int64_t kb = (int64_t)blockIdx.z * rows_per_split;
  int64_t ke = kb + rows_per_split;
  if (ke > n) ke = n;
  for (int64_t k0 = kb; k0 < ke; k0 += kGramRows) {
    __syncthreads();
    for (int e = t; e < kGramRows * 64; e += 256) {
      const int r = e / 64, c = e % 64;
      const int64_t k = k0 + r;
      xi_s[r][c] = (k < ke && ci0 + c < l) ? X[k * ldx + ci0 + c] : 0.0f;
      xj_s[r][c] = (k < ke && cj0 + c < l) ? X[k * ldx + cj0 + c] : 0.0f;
    }
    __syncthreads();
#pragma unroll 4
    for (int st = 0; st < kGramRows / 4; ++st) {
      const int r = 4 * st + lk;
      const double av = (double)xi_s[r][16 * w + li];
#pragma unroll
      for (int c = 0; c < 4; ++c)
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, (double)xj_s[r][16 * c + li], acc[c], 0, 0, 0);
    }
  }
  double *o = part + (int64_t)blockIdx.z * lp * lp;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int v = 0; v < 4; ++v) o[(ci0 + 16 * w + 4 * v + lk) * lp + cj0 + 16 * c + li] = acc[c][v];
}

__global__ void gram_big_reduce_kernel(const double *__restrict__ part, int nsplit, int64_t l,
                                       int64_t lp, double *__restrict__ K) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= l * l) return;
  int64_t i = e / l, j = e % l;
  if (i / 64 > j / 64) { const int64_t s = i; i = j; j = s; }   // read the upper tile
  double s = 0.0;
  for (int q = 0; q < nsplit; ++q) s += part[(int64_t)q * lp * lp + i * lp + j];
  K[e] = s;
}

static int gram_big_split(int64_t n, int64_t l) {
  const int64_t lp = (l + 63) / 64 * 64;
  const int64_t tiles = (lp / 64) * (lp / 64 + 1) / 2;
  int64_t s = (1024 + tiles - 1) / tiles;
  if (s > n / 256) s = n / 256;
  const int64_t cap = (int64_t)(256ll << 20) / (lp * lp * 8);   // partials <= 256 MiB
  if (s > cap) s = cap;
  if (s > 32) s = 32;
  if (s < 1) s = 1;
  return (int)s;
}

size_t gram_big_workspace_bytes(int64_t n, int64_t l) {
  const int64_t lp = (l + 63) / 64 * 64;
  return (size_t)gram_big_split(n, l) * lp * lp * 8;   // >= one full partial
}

void launch_gram_big(const float *X, int64_t ldx, int64_t n, int64_t l, double *K, void *work,
                     size_t work_bytes, hipStream_t st) {
  const int64_t lp = (l + 63) / 64 * 64;
  int s = gram_big_split(n, l);
  const int64_t fit = (int64_t)(work_bytes / ((size_t)lp * lp * 8));
  if (s > fit) s = (int)(fit < 1 ? 1 : fit);
  int64_t rows = (n + s - 1) / s;
  rows = (rows + kGramRows - 1) / kGramRows * kGramRows;
  const int ns = (int)((n + rows - 1) / rows);
  double *part = static_cast<double *>(work);
  dim3 grid((unsigned)(lp / 64), (unsigned)(lp / 64), (unsigned)ns);
  hipLaunchKernelGGL(gram_big_kernel, grid, dim3(256), 0, st, X, ldx, n, l, lp, rows, part);
  hipLaunchKernelGGL(gram_big_reduce_kernel, dim3((unsigned)((l * l + 255) / 256)), dim3(256), 0, st,
                     part, ns, l, lp, K);
}

// Y[r][c] = (float)(X[r][c] * f(c)), f = 1 or 1/s[c] (0 where s[c] == 0).
__global__ void convert_kernel(const double *__restrict__ X, int64_t rows, int64_t cols, int64_t ldx,
                               const double *__restrict__ s, float *__restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t r = e / cols, c = e % cols;
  double f = 1.0;
  if (s) f = (s[c] > 0.0) ? 1.0 / s[c] : 0.0;
  Y[r * ldy + c] = (float)(X[r * ldx + c] * f);
}

void launch_convert_f64_f32(const double *X, int64_t rows, int64_t cols, int64_t ldx,
                            const double *s, float *Y, int64_t ldy, hipStream_t st) {
  const int64_t tot = rows * cols;
  hipLaunchKernelGGL(convert_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, rows,
                     cols, ldx, s, Y, ldy);
}

__global__ void sqrt_clip_kernel(const double *__restrict__ w, int64_t l, double *__restrict__ s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < l) s[i] = w[i] > 0.0 ? sqrt(w[i]) : 0.0;
}

// Truncation rank of the fixed-precision output (Section 5.4 post-processing):
// scal[0] = ||A||_F^2, scal[1] = E; s (k values, descending).  The smallest r
// with E + sum_{i >= r} s_i^2 < tol^2 ||A||_F^2, the sum accumulated from the
// smallest value up and the scan stopped at the first r that fails; k when
// E itself fails or when `fixed` (fixed-rank use).  One thread: k <= l_max.
__global__ void trunc_rank_kernel(const double *__restrict__ s, int64_t k,
                                  const double *__restrict__ scal, double tol, int fixed,
                                  int64_t *__restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double thr = tol * tol * scal[0], e = scal[1];
  int64_t r = k;
  if (!fixed && e < thr) {
    double tail = 0.0;
    for (int64_t i = k - 1; i >= 0; --i) {
      tail += s[i] * s[i];
      if (e + tail < thr) r = i;
      else break;
    }
  }
  out[0] = r;
}

void launch_trunc_rank(const double *s, int64_t k, const double *scal, double tol, bool fixed,
                       int64_t *out, hipStream_t st) {
  hipLaunchKernelGGL(trunc_rank_kernel, dim3(1), dim3(64), 0, st, s, k, scal, tol, fixed ? 1 : 0, out);
}

void launch_sqrt_clip(const double *w, int64_t l, double *s, hipStream_t st) {
  hipLaunchKernelGGL(sqrt_clip_kernel, dim3((unsigned)((l + 255) / 256)), dim3(256), 0, st, w, l, s);
}

}  // namespace farpca_int
