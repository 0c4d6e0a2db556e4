// The product C_j^T = A^T Q_j with FP64 accumulation, for the indicator
// E = ||A||_F^2 - sum_j ||C_j||_F^2 (Algorithm 1; stop test of Section 5.2).
//
// The FP32 A-pass accumulates m products per entry in FP32, so ||C_j||_F^2
// carries a relative error of roughly 1e-8 .. 1e-7 and E, a difference of
// nearly equal sums, cannot resolve tol^2 ||A||^2 once tol^2 falls to that
// level (tol = 1e-4 asks for 1e-8).  Here every product of FP32 (or BF16)
// data is formed and summed in FP64 on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64): the products are exact and the sums carry FP64
// rounding, so ||C_j||^2 is known to the FP32 rounding of the basis itself.
//
// Layout: a workgroup (4 waves) owns 64 rows i of C^T (columns of A) and all
// 64 columns c; per 32-deep chunk of k it stages A (32 k x 64 i) and Q_j
// (32 k x 64 c) in LDS as FP64, and wave w accumulates rows 16 w .. 16 w + 15
// against the four 16-wide column tiles.  The k range is split over
// workgroups; FP64 partials (split x M x 64) are summed in split order by the
// finishing kernel, which also writes C^T in FP32 and the squared norm
// partials of the indicator.
#include "internal.h"

namespace farpca_int {

namespace {

constexpr int kC64Rows = 64;      // rows i per workgroup
constexpr int kC64K = 32;         // k per staged chunk
constexpr int kC64Ld = 66;        // LDS row stride (doubles)
constexpr int kC64Threads = 256;

typedef double doublex4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double widen64(float x) { return (double)x; }
__device__ __forceinline__ double widen64(uint16_t x) {
  return (double)__uint_as_float((uint32_t)x << 16);
}

// COLMAJOR: A is stored as A^T row-major (n x m, lda >= m): element (k, i) of
// A is A[i * lda + k].  Otherwise A is row-major (m x n): element (k, i) is
// A[k * lda + i].
template <typename T, bool COLMAJOR>
__global__ __launch_bounds__(kC64Threads) void cpass64_kernel(
    const T *__restrict__ A, int64_t lda, const float *__restrict__ Q, int64_t ldq, int64_t M,
    int64_t K, int64_t chunks_per_split, int64_t itiles, double *__restrict__ part) {
  __shared__ double al[kC64K * kC64Ld];
  __shared__ double ql[kC64K * kC64Ld];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t tile = blockIdx.x % itiles, split = blockIdx.x / itiles;
  const int64_t i0 = tile * kC64Rows;
  const int64_t kc0 = split * chunks_per_split;
  const int64_t nkc = (K + kC64K - 1) / kC64K;
  int64_t kc1 = kc0 + chunks_per_split;
  if (kc1 > nkc) kc1 = nkc;
  doublex4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = doublex4{0.0, 0.0, 0.0, 0.0};
  for (int64_t kc = kc0; kc < kc1; ++kc) {
    const int64_t k0 = kc * kC64K;
    if (COLMAJOR) {
      // 64 rows i of A^T, 32 contiguous k each: thread t takes row t / 4, k (t % 4) * 8 .. + 7
      const int r = tid >> 2, kk = (tid & 3) * 8;
      const int64_t i = i0 + r;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t k = k0 + kk + e;
        al[(kk + e) * kC64Ld + r] = (i < M && k < K) ? widen64(A[i * lda + k]) : 0.0;
      }
    } else {
      // 32 rows k of A, 64 contiguous i each: thread t takes row t / 8, i (t % 8) * 8 .. + 7
      const int kk = tid >> 3, r = (tid & 7) * 8;
      const int64_t k = k0 + kk;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t i = i0 + r + e;
        al[kk * kC64Ld + r + e] = (i < M && k < K) ? widen64(A[k * lda + i]) : 0.0;
      }
    }
    {
      const int kk = tid >> 3, c = (tid & 7) * 8;
      const int64_t k = k0 + kk;
#pragma unroll
      for (int e = 0; e < 8; ++e) ql[kk * kC64Ld + c + e] = k < K ? (double)Q[k * ldq + c + e] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kC64K / 4; ++ks) {
      const int kr = 4 * ks + (lane >> 4);
      const double av = al[kr * kC64Ld + 16 * w + (lane & 15)];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const double bv = ql[kr * kC64Ld + 16 * ct + (lane & 15)];
        acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ct], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // element v of acc[ct]: row 16 w + 4 v + lane / 16, column 16 ct + lane % 16
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t i = i0 + 16 * w + 4 * v + (lane >> 4);
    if (i >= M) continue;
    double *o = part + (split * M + i) * (int64_t)kBld;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) o[16 * ct + (lane & 15)] = acc[ct][v];
  }
}

// C[i, c] = sum over splits (in order) of part; C (FP32, ldc) for c < b;
// sq[g] = sum of C[i, c]^2 in FP64 (before rounding) over the rows of
// workgroup g (the partition of the FP32 squared norm, so the indicator sums
// the same number of partials).
__global__ __launch_bounds__(256) void cpass64_finish_kernel(const double *__restrict__ part, int nsplit,
                                                             int64_t M, int b, int64_t rows_per_wg,
                                                             float *__restrict__ C, int64_t ldc,
                                                             double *__restrict__ sq) {
  __shared__ double ws[4];
  const int t = threadIdx.x, c = t & 63;
  const int64_t rb = (int64_t)blockIdx.x * rows_per_wg;
  int64_t re = rb + rows_per_wg;
  if (re > M) re = M;
  double q = 0.0;
  for (int64_t r = rb + (t >> 6); r < re; r += 4) {
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) s += part[(sp * M + r) * (int64_t)kBld + c];
    if (c < b) {
      C[r * ldc + c] = (float)s;
      q = fma(s, s, q);
    }
  }
  q = wave_sum64(q);
  if ((t & 63) == 0) ws[t >> 6] = q;
  __syncthreads();
  if (t == 0) sq[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

}  // namespace

int cpass64_choose_split(int64_t M, int64_t K, int64_t max_split) {
  const int64_t itiles = (M + kC64Rows - 1) / kC64Rows;
  const int64_t nkc = (K + kC64K - 1) / kC64K;
  int64_t s = (1024 + itiles - 1) / itiles;        // about 4 workgroups per compute unit
  if (s > max_split) s = max_split;
  if (s > nkc) s = nkc;
  if (s < 1) s = 1;
  return (int)s;
}

void launch_cpass64(const void *A, bool bf16, bool colmajor, int64_t lda, const float *Q, int64_t ldq,
                    int64_t M, int64_t K, int b, int nsplit, double *part, float *C, int64_t ldc,
                    double *sq, hipStream_t st) {
  if (M <= 0) return;
  const int64_t itiles = (M + kC64Rows - 1) / kC64Rows;
  const int64_t nkc = (K + kC64K - 1) / kC64K;
  if (nsplit < 1) nsplit = 1;
  const int64_t cps = (nkc + nsplit - 1) / nsplit;
  nsplit = (int)((nkc + cps - 1) / cps);
  if (nsplit < 1) nsplit = 1;
  const dim3 grid((unsigned)(itiles * nsplit)), blk(kC64Threads);
  if (colmajor)
    hipLaunchKernelGGL((cpass64_kernel<float, true>), grid, blk, 0, st, static_cast<const float *>(A), lda, Q,
                       ldq, M, K, cps, itiles, part);
  else if (bf16)
    hipLaunchKernelGGL((cpass64_kernel<uint16_t, false>), grid, blk, 0, st, static_cast<const uint16_t *>(A),
                       lda, Q, ldq, M, K, cps, itiles, part);
  else
    hipLaunchKernelGGL((cpass64_kernel<float, false>), grid, blk, 0, st, static_cast<const float *>(A), lda, Q,
                       ldq, M, K, cps, itiles, part);
  const int64_t rows = (M + 255) / 256;
  const int nwg = (int)((M + rows - 1) / rows);
  hipLaunchKernelGGL(cpass64_finish_kernel, dim3(nwg), dim3(256), 0, st, part, nsplit, M, b, rows, C, ldc, sq);
}

}  // namespace farpca_int
