// Tall-skinny FP32 products on the CDNA matrix cores (v_mfma_f32_16x16x4_f32,
// FP32 accumulation): the dense A-passes of the power iteration and block
// products (Algorithm 1/2: A G_j and A^T Y_j) and the small basis products.
//
//   NN: C[M x N] = A[M x K] X[K x N]        (A row-major, reduce along a row)
//   TN: C[M x N] = A^T Y, A is K x M        (A row-major, reduce over rows)
// N <= 64 (one block of the method).  A workgroup = 4 waves owns a 64 x 64
// output tile; the 4 waves take interleaved 16-deep slices of K and their
// accumulators are summed through LDS in a fixed order.  Grid dimension y
// splits K further (partial tiles + reduce_partials) when the output alone
// has too few tiles to fill 256 CUs.
//
// Operand trick: a dot product may visit K in any order as long as both
// operands use the same order.  In NN each lane loads 4 consecutive K values
// of one A row with one 16-byte load and feeds them to 4 successive MFMAs
// (K slot l/16 of MFMA t <-> k = k0 + 4 (l/16) + t); X is read with the same
// mapping.  In TN each lane loads 4 consecutive columns of one A row (16
// bytes); component t feeds MFMA t, whose 16 output rows are then the
// columns c0 + 4 i + t (an interleaved output tile).
//
// MFMA 16x16x4 f32 operand layout (wave64): A lane l = (row l%16, k l/16),
// B lane l = (k l/16, col l%16), D lane l element v = (row 4 (l/16) + v, col l%16).
#include "internal.h"

namespace farpca_int {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <bool VEC>
__device__ __forceinline__ float4 load4_guard(const float *__restrict__ p, int64_t idx, int64_t lim) {
  // p points at element idx of a row with `lim` valid entries.
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (VEC && idx + 3 < lim) {
    v = *reinterpret_cast<const float4 *>(p);
  } else {
    if (idx + 0 < lim) v.x = p[0];
    if (idx + 1 < lim) v.y = p[1];
    if (idx + 2 < lim) v.z = p[2];
    if (idx + 3 < lim) v.w = p[3];
  }
  return v;
}

__device__ __forceinline__ float comp(const float4 &v, int t) {
  return t == 0 ? v.x : (t == 1 ? v.y : (t == 2 ? v.z : v.w));
}

// Sum the 4 waves' 64x64 accumulators (acc[16] floatx4 per lane) into wave 0.
__device__ __forceinline__ void wave_reduce(floatx4 (&acc)[16], float *red, int wave, int lane) {
  if (wave > 0) {
    float *dst = red + (wave - 1) * (16 * 4 * 64);
#pragma unroll
    for (int q = 0; q < 16; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) dst[(q * 4 + v) * 64 + lane] = acc[q][v];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const float *src = red + w * (16 * 4 * 64);
#pragma unroll
      for (int q = 0; q < 16; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[q][v] += src[(q * 4 + v) * 64 + lane];
    }
  }
}

// ---------------------------------------------------------------- NN
template <bool VEC>
__global__ __launch_bounds__(256) void gemm_nn_kernel(const float *__restrict__ A, int64_t lda,
                                                      const float *__restrict__ X, int64_t ldx,
                                                      float *__restrict__ C, int64_t ldc,
                                                      int64_t M, int64_t N, int64_t K,
                                                      int64_t k_per_split, float alpha, float beta,
                                                      float *__restrict__ part) {
  __shared__ float red[3 * 16 * 4 * 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  const int64_t kb = (int64_t)blockIdx.y * k_per_split;
  int64_t ke = kb + k_per_split;
  if (ke > K) ke = K;
  const int li = lane & 15, lk = lane >> 4;

  floatx4 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int64_t k0 = kb + 16 * wave; k0 < ke; k0 += 64) {
    const int64_t kk = k0 + 4 * lk;
    float4 a[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int64_t row = row0 + 16 * rt + li;
      a[rt] = (row < M) ? load4_guard<VEC>(A + row * lda + kk, kk, ke) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float x[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int64_t k = kk + t;
        const int64_t col = 16 * ct + li;
        x[t][ct] = (k < ke && col < N) ? X[k * ldx + col] : 0.0f;
      }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt * 4 + ct] = mfma4(comp(a[rt], t), x[t][ct], acc[rt * 4 + ct]);
  }
  wave_reduce(acc, red, wave, lane);
  if (wave != 0) return;
  // acc[rt*4+ct] element v: row = row0 + 16 rt + 4 lk + v, col = 16 ct + li
  float *dst = part ? part + (int64_t)blockIdx.y * M * kBld : C;
  const int64_t ld = part ? kBld : ldc;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + 16 * rt + 4 * lk + v;
        const int64_t col = 16 * ct + li;
        if (row < M && col < N) {
          float r = acc[rt * 4 + ct][v];
          if (!part) {
            r *= alpha;
            if (beta != 0.0f) r += beta * dst[row * ld + col];
          }
          dst[row * ld + col] = r;
        }
      }
}

// ---------------------------------------------------------------- TN
template <bool VEC>
__global__ __launch_bounds__(256) void gemm_tn_kernel(const float *__restrict__ A, int64_t lda,
                                                      const float *__restrict__ Y, int64_t ldy,
                                                      float *__restrict__ C, int64_t ldc,
                                                      int64_t M, int64_t N, int64_t K,
                                                      int64_t k_per_split, float alpha, float beta,
                                                      float *__restrict__ part) {
  __shared__ float red[3 * 16 * 4 * 64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  const int64_t kb = (int64_t)blockIdx.y * k_per_split;
  int64_t ke = kb + k_per_split;
  if (ke > K) ke = K;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t col_a = c0 + 4 * li;   // first of the 4 A columns this lane loads

  floatx4 acc[16];   // acc[t*4+ct]
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int64_t k0 = kb + 16 * wave; k0 < ke; k0 += 64) {
    float4 a[4];
    float y[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t k = k0 + 4 * q + lk;
      a[q] = (k < ke) ? load4_guard<VEC>(A + k * lda + col_a, col_a, M) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int64_t col = 16 * ct + li;
        y[q][ct] = (k < ke && col < N) ? Y[k * ldy + col] : 0.0f;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[t * 4 + ct] = mfma4(comp(a[q], t), y[q][ct], acc[t * 4 + ct]);
  }
  wave_reduce(acc, red, wave, lane);
  if (wave != 0) return;
  // acc[t*4+ct] element v: MFMA row i = 4 lk + v <-> output row c0 + 4 i + t, col 16 ct + li
  float *dst = part ? part + (int64_t)blockIdx.y * M * kBld : C;
  const int64_t ld = part ? kBld : ldc;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = c0 + 4 * (4 * lk + v) + t;
        const int64_t col = 16 * ct + li;
        if (row < M && col < N) {
          float r = acc[t * 4 + ct][v];
          if (!part) {
            r *= alpha;
            if (beta != 0.0f) r += beta * dst[row * ld + col];
          }
          dst[row * ld + col] = r;
        }
      }
}

// ---------------------------------------------------------------- reduce
__global__ void reduce_partials_kernel(const float *__restrict__ part, int nsplit, int64_t M,
                                       int64_t N, float *__restrict__ C, int64_t ldc, float alpha,
                                       float beta, const float *__restrict__ D, int64_t ldd,
                                       float gamma, const float *__restrict__ z, float zc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = idx / 64, col = idx % 64;
  if (row >= M || col >= N) return;
  float s = 0.0f;
  for (int q = 0; q < nsplit; ++q) s += part[((int64_t)q * M + row) * kBld + col];
  float r = alpha * s;
  if (beta != 0.0f) r += beta * C[row * ldc + col];
  if (D) r += gamma * D[row * ldd + col];
  if (z) r += zc * z[row];
  C[row * ldc + col] = r;
}

void launch_reduce_partials(const float *part, int nsplit, int64_t M, int64_t N, float *C,
                            int64_t ldc, float alpha, float beta, const float *D, int64_t ldd,
                            float gamma, const float *z, float zc, hipStream_t st) {
  const int64_t total = M * 64;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     part, nsplit, M, N, C, ldc, alpha, beta, D, ldd, gamma, z, zc);
}

int gemm_choose_ksplit(int64_t M, int64_t K, int /*is_tn*/) {
  const int64_t tiles = (M + 63) / 64;
  int64_t s = (1024 + tiles - 1) / tiles;       // about 1024 workgroups (4 waves each)
  const int64_t maxs = K / 256;                 // keep >= 256 K per split
  if (s > maxs) s = maxs;
  if (s > 8) s = 8;
  if (s < 1) s = 1;
  return (int)s;
}

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

void launch_gemm_nn(const float *A, int64_t lda, const float *X, int64_t ldx, float *C,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                    int ksplit, float *part, hipStream_t st) {
  if (ksplit < 1) ksplit = 1;
  int64_t kps = (K + ksplit - 1) / ksplit;
  kps = (kps + 63) / 64 * 64;
  const int nsp = (int)((K + kps - 1) / kps);
  float *p = (nsp > 1) ? part : nullptr;
  dim3 grid((unsigned)((M + 63) / 64), (unsigned)nsp);
  const bool vec = (lda % 4 == 0) && aligned16(A);
  if (vec) hipLaunchKernelGGL((gemm_nn_kernel<true>), grid, dim3(256), 0, st, A, lda, X, ldx, C, ldc,
                              M, N, K, kps, alpha, beta, p);
  else hipLaunchKernelGGL((gemm_nn_kernel<false>), grid, dim3(256), 0, st, A, lda, X, ldx, C, ldc,
                          M, N, K, kps, alpha, beta, p);
  if (nsp > 1) launch_reduce_partials(part, nsp, M, N, C, ldc, alpha, beta, nullptr, 0, 0.f,
                                      nullptr, 0.f, st);
}

void launch_gemm_tn(const float *A, int64_t lda, const float *Y, int64_t ldy, float *C,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                    int ksplit, float *part, hipStream_t st) {
  if (ksplit < 1) ksplit = 1;
  int64_t kps = (K + ksplit - 1) / ksplit;
  kps = (kps + 63) / 64 * 64;
  const int nsp = (int)((K + kps - 1) / kps);
  float *p = (nsp > 1) ? part : nullptr;
  dim3 grid((unsigned)((M + 63) / 64), (unsigned)nsp);
  const bool vec = (lda % 4 == 0) && aligned16(A);
  if (vec) hipLaunchKernelGGL((gemm_tn_kernel<true>), grid, dim3(256), 0, st, A, lda, Y, ldy, C, ldc,
                              M, N, K, kps, alpha, beta, p);
  else hipLaunchKernelGGL((gemm_tn_kernel<false>), grid, dim3(256), 0, st, A, lda, Y, ldy, C, ldc,
                          M, N, K, kps, alpha, beta, p);
  if (nsp > 1) launch_reduce_partials(part, nsp, M, N, C, ldc, alpha, beta, nullptr, 0, 0.f,
                                      nullptr, 0.f, st);
}

}  // namespace farpca_int
