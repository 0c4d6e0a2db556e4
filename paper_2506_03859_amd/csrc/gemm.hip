// Tall-skinny FP32 products on the CDNA matrix cores (v_mfma_f32_16x16x4_f32,
// FP32 accumulation): the dense A-passes of the power iteration and block
// products (Algorithm 1/2: A G_j and A^T Y_j) and the small basis products.
//
//   NN: C[M x N] = A[M x K] X[K x N]        (A row-major, reduce along a row)
//   TN: C[M x N] = A^T Y, A is K x M        (A row-major, reduce over rows)
// N <= 64 (one block of the method); X / Y is the "skinny" operand.
//
// A workgroup has 4 waves.  Each wave accumulates one 64 x 64 output tile in
// registers.  Two layouts (template WM = waves along the output dimension):
//   WM = 4  the 4 waves own 4 consecutive output tiles (256 rows) and walk
//           the same K range: every staged skinny chunk feeds 4 tiles, so the
//           skinny operand costs a quarter of A's bytes (large M);
//   WM = 1  the 4 waves share one output tile and take interleaved 16-deep
//           K slices; their accumulators are summed through LDS in a fixed
//           order at the end (small M: more workgroups per output tile).
// Grid: tiles x K splits, flattened and remapped so that the workgroups of
// one K split run on the same XCD (consecutive logical ids share an L2 there
// and with it the skinny chunk).  With more than one split the kernel writes
// partial tiles and reduce_partials sums them in split order.
//
// Per 16-deep K slice a lane issues 4 16-byte loads of A (registers, fetched
// one chunk ahead), reads 16 skinny values from LDS and issues 64 MFMAs.  The
// skinny chunk is staged in LDS row-major (stride 68 floats: the 16-byte
// stores and the 4-byte reads are bank-conflict free), double buffered, one
// barrier per chunk.
//
// K order: a dot product may visit K in any order as long as both operands
// use the same one.  NN: lane (li = l%16, lk = l/16) loads 4 consecutive K
// values of A row 16 rt + li; component t feeds MFMA t, whose K slot lk is
// k = k0 + 4 lk + t.  TN: lane loads 4 consecutive A columns c0 + 4 li .. +3
// of A rows k0 + 4 lk + q; component t feeds MFMA (q, t), whose 16 output
// rows are then the columns c0 + 4 i + t (an interleaved output tile).  In
// both the skinny operand is read at chunk row 16 wk + 4 lk + u, column
// 16 ct + li.
//
// MFMA 16x16x4 f32 operand layout (wave64): A lane l = (row l%16, k l/16),
// B lane l = (k l/16, col l%16), D lane l element v = (row 4 (l/16) + v, col l%16).
#include <map>
#include <mutex>
#include <tuple>

#include "internal.h"

namespace farpca_int {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kXs = 68;   // floats per staged skinny row (64 + 4 pad)

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float comp(const float4 &v, int t) {
  return t == 0 ? v.x : (t == 1 ? v.y : (t == 2 ? v.z : v.w));
}

__device__ __forceinline__ int64_t clampi(int64_t v, int64_t hi) { return v < hi ? v : hi; }

// Logical workgroup id: physical ids g = 8 j + x run on XCD x; the first
// 8 floor(T/8) ids are regrouped so that XCD x gets a contiguous logical range.
__device__ __forceinline__ int64_t xcd_remap(int64_t g, int64_t T) {
  const int64_t T8 = T & ~int64_t(7);
  if (g >= T8) return g;
  return (g & 7) * (T8 >> 3) + (g >> 3);
}

// Per-lane A base pointer (the part of the address fixed for the whole K
// range).  Rows (NN) / columns (TN) outside M are clamped into the matrix:
// they only feed outputs that are never stored.
template <bool TN, bool AVEC>
__device__ __forceinline__ const float *a_base(const float *__restrict__ A, int64_t lda,
                                               int64_t M, int64_t t0, int li, int lk) {
  if (!TN) return A + 4 * lk;                       // + row * lda + k0 per load
  int64_t col = t0 + 4 * li;
  if (AVEC) col = col < M - 4 ? col : M - 4;        // AVEC: here M % 4 == 0, M >= 4
  return A + 4 * lk * lda + col;                    // + (k0 + q) * lda per load
}

// A-operand loads of one full 16-deep slice at k0 (inside K): 4 float4 per lane.
template <bool TN, bool AVEC>
__device__ __forceinline__ void load_a_full(const float *__restrict__ ab, int64_t lda, int64_t M,
                                            int64_t t0, int li, int64_t k0, float4 (&a)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float *p;
    if (!TN) {
      const int64_t row = clampi(t0 + 16 * q + li, M - 1);
      p = ab + row * lda + k0;
    } else {
      p = ab + (k0 + q) * lda;
    }
    if (AVEC) {
      a[q] = *reinterpret_cast<const float4 *>(p);
    } else if (!TN) {
      a[q] = make_float4(p[0], p[1], p[2], p[3]);
    } else {
      // scalar columns, each clamped into M (p is at column t0 + 4 li)
      const int64_t col = t0 + 4 * li;
      float v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) v[t] = p[clampi(col + t, M - 1) - col];
      a[q] = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
}

// The same for the last, partial slice: addresses clamped into [.., ke) and
// values beyond K zeroed (scalar loads).
template <bool TN>
__device__ __forceinline__ void load_a_tail(const float *__restrict__ A, int64_t lda, int64_t M,
                                            int64_t ke, int64_t t0, int li, int lk, int64_t k0,
                                            float4 (&a)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float v[4];
    if (!TN) {
      const float *p = A + clampi(t0 + 16 * q + li, M - 1) * lda;
      const int64_t kk = k0 + 4 * lk;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float u = p[clampi(kk + t, ke - 1)];
        v[t] = (kk + t < ke) ? u : 0.0f;
      }
    } else {
      const int64_t k = k0 + 4 * lk + q;
      const float *p = A + clampi(k, ke - 1) * lda;
      const int64_t col = t0 + 4 * li;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float u = p[clampi(col + t, M - 1)];
        v[t] = (k < ke) ? u : 0.0f;
      }
    }
    a[q] = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// Skinny chunk rows [kc, kc + 16 NX) into registers: thread tid holds float4
// number f = tid + 256 j (chunk row f / 16, columns 4 (f % 16) .. +3).
// XVEC (rows 16-byte aligned with 64 readable floats: N == 64 or ldx >= 64)
// and rows inside K: one 16-byte load, columns >= N set to zero (the last
// row of the range is read that way only when N == 64: a caller's buffer may
// end at its N-th column); otherwise clamped scalar loads, zero outside K x N.
// NN with WM = 4 (the A-passes A G): a wave's 64 rows x 32 K of a chunk are
// read as 8 rows x 128 contiguous bytes per instruction (lane l: row
// 8 q + l / 8, K 4 (l % 8) .. + 3) - twice the row piece of the MFMA operand
// layout, which the memory system serves faster - and regrouped through a
// wave-private LDS area into that layout: row r, K group g (4 floats) at
// r * 32 + 4 (g ^ (r % 8)); the XOR keeps both the 8-lane row writes and the
// 16-row column reads bank-conflict free without padding.
constexpr int kStageRowF = 32;   // floats per staged row (one chunk of K)
__device__ __forceinline__ int stage_off(int r, int g) { return r * kStageRowF + 4 * (g ^ (r & 7)); }

__device__ __forceinline__ void load_a_runs(const float *__restrict__ A, int64_t lda, int64_t M,
                                            int64_t t0, int lane, int64_t kc, float4 (&r)[2][4]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t row = clampi(t0 + 8 * q + (lane >> 3), M - 1);
    const floatx4 v = *reinterpret_cast<const floatx4 *>(A + row * lda + kc + 4 * (lane & 7));
    r[q >> 2][q & 3] = make_float4(v[0], v[1], v[2], v[3]);   // element copies: no struct memcpy
  }
}

__device__ __forceinline__ void stage_in(float *wst, int lane, const float4 (&r)[2][4]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float4 &v = r[q >> 2][q & 3];
    *reinterpret_cast<floatx4 *>(wst + stage_off(8 * q + (lane >> 3), lane & 7)) = floatx4{v.x, v.y, v.z, v.w};
  }
}

// The MFMA operand of slice s, row tile rt: row 16 rt + li, K 16 s + 4 lk .. + 3
// (the same values load_a_full reads for NN).
__device__ __forceinline__ void stage_out(const float *wst, int li, int lk, int s, float4 (&a)[4]) {
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    const floatx4 v = *reinterpret_cast<const floatx4 *>(wst + stage_off(16 * rt + li, 4 * s + lk));
    a[rt] = make_float4(v[0], v[1], v[2], v[3]);
  }
}

template <int NX, bool XVEC>
__device__ __forceinline__ void load_x(const float *__restrict__ X, int64_t ldx, int64_t N,
                                       int64_t ke, int64_t kc, int tid, bool full,
                                       float4 (&xr)[NX]) {
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    const int f = tid + 256 * j;
    const int64_t k = kc + (f >> 4);
    const int col = 4 * (f & 15);
    if (XVEC && full && (N == 64 || k + 1 < ke)) {
      float4 v = *reinterpret_cast<const float4 *>(X + k * ldx + col);
      if (N < 64) {
        v.x = col < N ? v.x : 0.0f;
        v.y = col + 1 < N ? v.y : 0.0f;
        v.z = col + 2 < N ? v.z : 0.0f;
        v.w = col + 3 < N ? v.w : 0.0f;
      }
      xr[j] = v;
    } else {
      const float *p = X + clampi(k, ke - 1) * ldx;
      float v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float u = p[clampi(col + t, N - 1)];
        v[t] = (k < ke && col + t < N) ? u : 0.0f;
      }
      xr[j] = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
}

template <int NX>
__device__ __forceinline__ void store_x(float *xs, int tid, const float4 (&xr)[NX]) {
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    const int f = tid + 256 * j;
    *reinterpret_cast<float4 *>(xs + (f >> 4) * kXs + 4 * (f & 15)) = xr[j];
  }
}

// 64 MFMAs of one 16-deep slice: skinny values from LDS rows 4 lk + u of
// the slice.
template <bool TN>
__device__ __forceinline__ void mma_slice(floatx4 (&acc)[16], const float4 (&a)[4],
                                          const float *xslice, int li, int lk) {
  const float *xb = xslice + 4 * lk * kXs + li;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    float xv[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) xv[ct] = xb[u * kXs + 16 * ct];
    if (!TN) {
      // NN: MFMA u takes component u of every row group rt
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          acc[rt * 4 + ct] = mfma4(comp(a[rt], u), xv[ct], acc[rt * 4 + ct]);
    } else {
      // TN: load u (A row k0 + 4 lk + u) feeds the 4 interleaved column groups t
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int ct = 0; ct < 4; ++ct)
          acc[t * 4 + ct] = mfma4(comp(a[u], t), xv[ct], acc[t * 4 + ct]);
    }
  }
}

// Occupancy: 3 blocks per CU, except the staged NN form, whose two register
// copies of a chunk plus the accumulators need up to 2 blocks' worth of VGPRs.
template <bool TN, int WM, bool AVEC, bool XVEC>
__global__ __launch_bounds__(256, (AVEC && (TN || WM != 4)) ? 3 : 2) void gemm_kernel(const float *__restrict__ A, int64_t lda,
                                                      const float *__restrict__ X, int64_t ldx,
                                                      float *__restrict__ C, int64_t ldc,
                                                      int64_t M, int64_t N, int64_t K,
                                                      int64_t kps, int64_t tiles, int64_t total,
                                                      int64_t mload,
                                                      float alpha, float beta,
                                                      float *__restrict__ part) {
  constexpr int WK = 4 / WM;
  constexpr int SL = (WM == 4) ? 2 : 1;   // 16-deep slices per wave per chunk
  constexpr int KW = 16 * SL;             // K rows per wave per chunk
  constexpr int KC = KW * WK;             // skinny rows per staged chunk
  constexpr int NX = KC / 16;             // skinny float4 loads per thread per chunk
  constexpr bool STAGE = !TN && WM == 4 && AVEC;
  static_assert(!STAGE || (SL == 2 && KC == kStageRowF), "staging covers one 32-deep chunk");
  __shared__ float xs[2][KC * kXs];
  __shared__ float ast[STAGE ? 4 * 64 * kStageRowF : 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave % WM, wk = wave / WM;
  const int li = lane & 15, lk = lane >> 4;

  const int64_t L = xcd_remap(blockIdx.x, total);
  const int64_t tile = L % tiles, split = L / tiles;
  const int64_t t0 = (tile * WM + wm) * 64;        // first output row of this wave's tile
  const int64_t kb = split * kps;
  const int64_t ke = (kb + kps < K) ? kb + kps : K;
  const int64_t nfull = (ke - kb) / KC;            // chunks entirely inside [kb, ke)
  // TN: 16-byte column loads are clamped into the first mload columns (M, or
  // M rounded up to 4 when the row padding up to lda may be read: its
  // columns only feed outputs that are never stored)
  const float *ab = a_base<TN, AVEC>(A, lda, TN ? mload : M, t0, li, lk);

  floatx4 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};

  // Chunk c: A slices in `cur`, skinny rows in xs[c & 1].  Chunk c + 1 is
  // fetched (A into `nxt`, skinny rows into `xr`) before the MFMAs of chunk
  // c; the scheduling barriers keep the compiler from sinking those loads
  // below the MFMAs, which would serialise memory latency and compute.
  // STAGE: `a` receives the 8 row pieces (row-piece layout), not MFMA operands
  float4 cur[SL][4], nxt[SL][4], xr[NX];
  float *wst = ast + (STAGE ? wave * 64 * kStageRowF : 0);
  auto fetch = [&](int64_t c, float4 (&a)[SL][4]) {
    const int64_t kc = kb + c * KC;
    load_x<NX, XVEC>(X, ldx, N, ke, kc, tid, true, xr);
    if constexpr (STAGE) {
      load_a_runs(A, lda, M, t0, lane, kc, a);
    } else {
#pragma unroll
      for (int s = 0; s < SL; ++s)
        load_a_full<TN, AVEC>(ab, lda, M, t0, li, kc + KW * wk + 16 * s, a[s]);
    }
  };
  auto mma_chunk = [&](int64_t c) {
#pragma unroll
    for (int s = 0; s < SL; ++s) mma_slice<TN>(acc, cur[s], xs[c & 1] + (KW * wk + 16 * s) * kXs, li, lk);
  };
  // STAGE: the staged chunk is read back into `cur` right after the
  // barrier (reading it slice by slice between the MFMAs measured slower)
  auto unstage = [&]() {
#pragma unroll
    for (int s = 0; s < SL; ++s) stage_out(wst, li, lk, s, cur[s]);
  };

  if (nfull > 0) {
    if constexpr (STAGE) {
      fetch(0, nxt);
      stage_in(wst, lane, nxt);
      unstage();
    } else {
      fetch(0, cur);
    }
    store_x<NX>(xs[0], tid, xr);
    __syncthreads();
    for (int64_t c = 0; c + 1 < nfull; ++c) {
      fetch(c + 1, nxt);
      __builtin_amdgcn_sched_barrier(0);
      mma_chunk(c);
      __builtin_amdgcn_sched_barrier(0);
      store_x<NX>(xs[(c + 1) & 1], tid, xr);
      // wave-private area: the wave's reads of chunk c precede these writes
      // in its own program order
      if constexpr (STAGE) stage_in(wst, lane, nxt);
      __syncthreads();
      if constexpr (STAGE) {
        unstage();
      } else {
#pragma unroll
        for (int s = 0; s < SL; ++s)
#pragma unroll
          for (int q = 0; q < 4; ++q) cur[s][q] = nxt[s][q];
      }
    }
    mma_chunk(nfull - 1);
    __syncthreads();
  }
  if (kb + nfull * KC < ke) {
    // the partial last chunk (every reader of xs has passed the last barrier)
    const int64_t kc = kb + nfull * KC;
    load_x<NX, false>(X, ldx, N, ke, kc, tid, false, xr);
#pragma unroll
    for (int s = 0; s < SL; ++s)
      load_a_tail<TN>(A, lda, M, ke, t0, li, lk, kc + KW * wk + 16 * s, cur[s]);
    store_x<NX>(xs[0], tid, xr);
    __syncthreads();
    mma_chunk(0);
    __syncthreads();
  }

  if (WK > 1) {
    // fixed-order sum of the 4 K-interleaved accumulators into wave 0:
    // (w0 + w2) + (w1 + w3), staged through the (now free) skinny buffers
    // (2 KC kXs >= 2 x 4096 floats)
    float *red = &xs[0][0];
    auto put = [&](int slot) {
#pragma unroll
      for (int q = 0; q < 16; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[slot * 4096 + (q * 4 + v) * 64 + lane] = acc[q][v];
    };
    auto add = [&](int slot) {
#pragma unroll
      for (int q = 0; q < 16; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[q][v] += red[slot * 4096 + (q * 4 + v) * 64 + lane];
    };
    if (wave >= 2) put(wave - 2);
    __syncthreads();
    if (wave < 2) add(wave);
    __syncthreads();
    if (wave == 1) put(0);
    __syncthreads();
    if (wave != 0) return;
    add(0);
  }

  float *dst = part ? part + split * M * kBld : C;
  const int64_t ld = part ? kBld : ldc;
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // NN: acc[rt*4+ct][v] -> row t0 + 16 rt + 4 lk + v
        // TN: acc[t*4+ct][v]  -> row t0 + 4 (4 lk + v) + t
        const int64_t row = TN ? t0 + 4 * (4 * lk + v) + g : t0 + 16 * g + 4 * lk + v;
        const int64_t col = 16 * ct + li;
        if (row < M && col < N) {
          float r = acc[g * 4 + ct][v];
          if (!part) {
            r *= alpha;
            if (beta != 0.0f) r += beta * dst[row * ld + col];
          }
          dst[row * ld + col] = r;
        }
      }
}

// ---------------------------------------------------------------- reduce
// C = alpha * (sum of the partial tiles in split order) [+ beta C] [+ gamma D]
// [+ zc z_row].  A thread owns 4 adjacent columns of a row: the partials are
// read with 16-byte loads when the buffer is 16-byte aligned (VEC; the tiles
// are 64 floats wide), the splits requested together; each element's
// arithmetic is the same as with one thread per element.
template <bool VEC>
__global__ __launch_bounds__(256) void reduce_partials_kernel(
    const float *__restrict__ part, int nsplit, int64_t M, int64_t N, float *__restrict__ C,
    int64_t ldc, float alpha, float beta, const float *__restrict__ D, int64_t ldd, float gamma,
    const float *__restrict__ z, float zc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = idx / 16;
  const int c4 = (int)(idx % 16) * 4;
  if (row >= M || c4 >= N) return;
  float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (VEC) {
    const float4 *p = reinterpret_cast<const float4 *>(part + row * kBld + c4);
    const int64_t stride = M * kBld / 4;               // one split, in float4
    int q = 0;
    for (; q + 4 <= nsplit; q += 4) {
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = p[(int64_t)(q + u) * stride];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        s[0] += v[u].x; s[1] += v[u].y; s[2] += v[u].z; s[3] += v[u].w;
      }
    }
    for (; q < nsplit; ++q) {
      const float4 v = p[(int64_t)q * stride];
      s[0] += v.x; s[1] += v.y; s[2] += v.z; s[3] += v.w;
    }
  } else {
    for (int q = 0; q < nsplit; ++q) {
      const float *pq = part + ((int64_t)q * M + row) * kBld + c4;
#pragma unroll
      for (int i = 0; i < 4; ++i) s[i] += pq[i];
    }
  }
  const float zr = z ? zc * z[row] : 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t col = c4 + i;
    if (col >= N) break;
    float r = alpha * s[i];
    if (beta != 0.0f) r += beta * C[row * ldc + col];
    if (D) r += gamma * D[row * ldd + col];
    if (z) r += zr;
    C[row * ldc + col] = r;
  }
}

void launch_reduce_partials(const float *part, int nsplit, int64_t M, int64_t N, float *C,
                            int64_t ldc, float alpha, float beta, const float *D, int64_t ldd,
                            float gamma, const float *z, float zc, hipStream_t st) {
  const int64_t total = M * 16;
  const dim3 grid((unsigned)((total + 255) / 256)), blk(256);
  if ((reinterpret_cast<uintptr_t>(part) & 15) == 0)
    hipLaunchKernelGGL(reduce_partials_kernel<true>, grid, blk, 0, st, part, nsplit, M, N, C, ldc,
                       alpha, beta, D, ldd, gamma, z, zc);
  else
    hipLaunchKernelGGL(reduce_partials_kernel<false>, grid, blk, 0, st, part, nsplit, M, N, C, ldc,
                       alpha, beta, D, ldd, gamma, z, zc);
}

void launch_gemm_finish(const float *part, int nsp, int64_t M, int64_t N, float *C, int64_t ldc,
                        float alpha, float beta, hipStream_t st) {
  if (nsp > 1) launch_reduce_partials(part, nsp, M, N, C, ldc, alpha, beta, nullptr, 0, 0.f,
                                      nullptr, 0.f, st);
}

// Workgroups of the aligned kernel for (TN, WM) that are resident on the
// current device at once (compute units x occupancy); queried once per device.
static int64_t gemm_slots(int is_tn, int wm) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int>, int64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(dev, is_tn, wm);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  const void *fn = is_tn ? (wm == 4 ? reinterpret_cast<const void *>(&gemm_kernel<true, 4, true, true>)
                                    : reinterpret_cast<const void *>(&gemm_kernel<true, 1, true, true>))
                         : (wm == 4 ? reinterpret_cast<const void *>(&gemm_kernel<false, 4, true, true>)
                                    : reinterpret_cast<const void *>(&gemm_kernel<false, 1, true, true>));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0) != hipSuccess || per_cu < 1)
    per_cu = 2;
  const int64_t slots = (int64_t)cus * per_cu;
  cache[key] = slots;
  return slots;
}

// Modelled time of the layout WM with sp K splits, in units of one wave's
// MFMA work on one 64-row tile per K row: rounds of resident workgroups x the
// K rows each wave walks (K / sp, or K / (4 sp) when the four waves
// interleave K) x the cost of the partial tiles (written and read once more)
// x the bytes staged per byte of A (the skinny chunk feeds 4 tiles at WM = 4,
// one at WM = 1) x the padding of the last tile.
static double gemm_cost(int64_t M, int64_t K, int wm, int64_t sp, int64_t slots) {
  const int64_t tiles = (M + 64 * wm - 1) / (64 * wm);
  const int64_t rounds = (tiles * sp + slots - 1) / slots;
  const double depth = (double)K / (double)sp / (wm == 4 ? 1.0 : 4.0);
  const double staged = wm == 4 ? 1.25 : 2.0;
  const double pad = (double)(tiles * 64 * wm) / (double)M;
  return (double)rounds * depth * (1.0 + 128.0 * (double)sp / (double)K) * staged * pad;
}

// Best split count of layout wm for at most smax splits (and its cost).
static int gemm_best_split(int64_t M, int64_t K, int wm, int64_t smax, int64_t slots, double *cost) {
  if (smax > K / 256) smax = K / 256;
  if (smax > 64) smax = 64;
  if (smax < 1) smax = 1;
  int best = 1;
  double best_cost = 0.0;
  for (int64_t sp = 1; sp <= smax; ++sp) {
    const double c = gemm_cost(M, K, wm, sp, slots);
    if (sp == 1 || c < best_cost * (1.0 - 1e-9)) {
      best = (int)sp;
      best_cost = c;
    }
  }
  if (cost) *cost = best_cost;
  return best;
}

// Waves along the output dimension: the cheaper layout under the model
// (short products, K < 1024 - the basis products Q r, K = l - always take
// WM = 1).  The choice does not depend on the caller's split limit, so that
// launch and split choice agree.
static int gemm_wm(int64_t M, int64_t K, int is_tn) {
  // short NN products (Q r: K = l) past kShortMaxM rows (below it they take
  // gemm_nn_short_kernel): each wave walks the whole K range of its own 64
  // rows (no cross-wave reduction at the end)
  if (K < 1024) return (!is_tn && M >= 131072) ? 4 : 1;
  double c1 = 0.0, c4 = 0.0;
  gemm_best_split(M, K, 1, 64, gemm_slots(is_tn, 1), &c1);
  gemm_best_split(M, K, 4, 64, gemm_slots(is_tn, 4), &c4);
  return c4 < c1 ? 4 : 1;
}

// Number of K splits for the chosen layout: all workgroups in as few rounds
// of resident workgroups as possible, each split at least 256 K rows, the
// partial tiles cheap next to A.
int gemm_choose_ksplit(int64_t M, int64_t K, int is_tn, int64_t max_split) {
  if (M < 1 || K < 1) return 1;
  const int wm = gemm_wm(M, K, is_tn);
  return gemm_best_split(M, K, wm, max_split, gemm_slots(is_tn, wm), nullptr);
}

static bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// ------------------------------------------------------------- short K (NN)
// The basis products Q r (K = l, a few hundred) are latency-bound in the
// chunk pipeline above (one DRAM round trip per 64-deep chunk, 15-25 us per
// launch against a few us of HBM time).  Here a workgroup of 8 waves owns 128
// output rows; every wave issues the loads of its 16 rows over the whole K at
// once (one 16-byte load per 16-deep slice and lane, at most kShortK / 16
// slices in registers), the workgroup stages all of X (K x 64) in LDS, and
// after one barrier each wave runs its K / 4 steps of 4 MFMAs.  Same MFMA
// operand order as gemm_kernel (lane (li, lk), slice s: row li, k = 16 s +
// 4 lk + u for MFMA u).
constexpr int kShortK = 384;
// The X stage takes 104 KB of LDS (one workgroup per CU): past about 130000
// rows (over 4 rounds of workgroups) the 4-tile chunk pipeline is faster.
constexpr int64_t kShortMaxM = 131072;
constexpr int kShortWaves = 8;
constexpr int kShortRows = 16 * kShortWaves;

template <bool AVEC, bool XVEC>
__global__ __launch_bounds__(64 * kShortWaves) void gemm_nn_short_kernel(
    const float *__restrict__ A, int64_t lda, const float *__restrict__ X, int64_t ldx,
    float *__restrict__ C, int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta) {
  constexpr int kMaxSl = kShortK / 16;
  __shared__ float xs[kShortK * kXs];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nsl = (int)((K + 15) / 16);
  const int64_t r0 = (int64_t)blockIdx.x * kShortRows + 16 * wave;
  const float *ar = A + clampi(r0 + li, M - 1) * lda;
  float4 a[kMaxSl];
#pragma unroll
  for (int s = 0; s < kMaxSl; ++s) {
    if (s < nsl) {
      const int64_t g = 16 * s + 4 * lk;
      if (AVEC && g + 4 <= K) {
        a[s] = *reinterpret_cast<const float4 *>(ar + g);
      } else {
        float v[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float u = ar[clampi(g + t, K - 1)];
          v[t] = (g + t < K) ? u : 0.0f;
        }
        a[s] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  }
  // X rows 0 .. 16 nsl - 1 (zero past K and past column N)
  const int nf = 16 * 16 * nsl;                  // float4 pieces
  for (int f = tid; f < nf; f += 64 * kShortWaves) {
    const int64_t k = f >> 4;
    const int col = 4 * (f & 15);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (k < K) {
      // the last row is read by vector only when N == 64: a caller's buffer
      // may end at its N-th column
      if (XVEC && (N == 64 || k + 1 < K)) {
        v = *reinterpret_cast<const float4 *>(X + k * ldx + col);
        if (N < 64) {
          v.x = col < N ? v.x : 0.0f;
          v.y = col + 1 < N ? v.y : 0.0f;
          v.z = col + 2 < N ? v.z : 0.0f;
          v.w = col + 3 < N ? v.w : 0.0f;
        }
      } else {
        const float *p = X + k * ldx;
        float w[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const float u = p[clampi(col + t, N - 1)];
          w[t] = (col + t < N) ? u : 0.0f;
        }
        v = make_float4(w[0], w[1], w[2], w[3]);
      }
    }
    *reinterpret_cast<float4 *>(xs + k * kXs + col) = v;
  }
  __syncthreads();
  floatx4 acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < kMaxSl; ++s) {
    if (s < nsl) {
      const float *xb = xs + (16 * s + 4 * lk) * kXs + li;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float av = comp(a[s], u);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma4(av, xb[u * kXs + 16 * ct], acc[ct]);
      }
    }
  }
  // D lane l element v = (row 4 (l / 16) + v, column l % 16)
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 4 * lk + v;
      const int64_t col = 16 * ct + li;
      if (row < M && col < N) {
        float r = alpha * acc[ct][v];
        if (beta != 0.0f) r += beta * C[row * ldc + col];
        C[row * ldc + col] = r;
      }
    }
}

template <bool TN>
static int launch_main(const float *A, int64_t lda, const float *X, int64_t ldx, float *C,
                       int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                       int ksplit, float *part, hipStream_t st) {
  if (M <= 0 || N <= 0) return 1;
  if (ksplit < 1) ksplit = 1;
  if (!TN && K > 0 && K <= kShortK && M < kShortMaxM) {
    const bool avec = (lda % 4 == 0) && aligned16(A);
    const bool xvec = (ldx % 4 == 0) && aligned16(X) && (N == 64 || ldx >= 64);
    const dim3 grid((unsigned)((M + kShortRows - 1) / kShortRows)), blk(64 * kShortWaves);
#define FARPCA_SHORT_LAUNCH(AV, XV)                                                               \
  hipLaunchKernelGGL((gemm_nn_short_kernel<AV, XV>), grid, blk, 0, st, A, lda, X, ldx, C, ldc, M, N, \
                     K, alpha, beta)
    if (avec && xvec) FARPCA_SHORT_LAUNCH(true, true);
    else if (avec) FARPCA_SHORT_LAUNCH(true, false);
    else if (xvec) FARPCA_SHORT_LAUNCH(false, true);
    else FARPCA_SHORT_LAUNCH(false, false);
#undef FARPCA_SHORT_LAUNCH
    return 1;
  }
  const int wm = gemm_wm(M, K, TN ? 1 : 0);
  const int64_t kc = (wm == 4) ? 32 : 64;        // K rows per chunk (KC)
  int64_t kps = (K + ksplit - 1) / ksplit;
  kps = (kps + 63) / 64 * 64;                    // whole chunks per split
  if (kps < kc) kps = kc;
  const int nsp = K > 0 ? (int)((K + kps - 1) / kps) : 1;
  float *p = (nsp > 1) ? part : nullptr;
  const int64_t tiles = (M + 64 * wm - 1) / (64 * wm);
  const int64_t total = tiles * nsp;
  const int64_t m4 = (M + 3) / 4 * 4;
  const int64_t mload = (M % 4 == 0) ? M : (m4 <= lda ? m4 : 0);
  const bool avec = (lda % 4 == 0) && aligned16(A) && (!TN || mload >= 4);
  const bool xvec = (ldx % 4 == 0) && aligned16(X) && (N == 64 || ldx >= 64);
  dim3 grid((unsigned)total), blk(256);
#define FARPCA_GEMM_LAUNCH(WMV, AV, XV)                                                            \
  hipLaunchKernelGGL((gemm_kernel<TN, WMV, AV, XV>), grid, blk, 0, st, A, lda, X, ldx, C, ldc, M, \
                     N, K, kps, tiles, total, mload, alpha, beta, p)
#define FARPCA_GEMM_LAUNCH_WM(WMV)                  \
  do {                                              \
    if (avec && xvec) FARPCA_GEMM_LAUNCH(WMV, true, true);          \
    else if (avec) FARPCA_GEMM_LAUNCH(WMV, true, false);            \
    else if (xvec) FARPCA_GEMM_LAUNCH(WMV, false, true);            \
    else FARPCA_GEMM_LAUNCH(WMV, false, false);                     \
  } while (0)
  if (wm == 4) FARPCA_GEMM_LAUNCH_WM(4);
  else FARPCA_GEMM_LAUNCH_WM(1);
#undef FARPCA_GEMM_LAUNCH_WM
#undef FARPCA_GEMM_LAUNCH
  return nsp;
}

int launch_gemm_nn_main(const float *A, int64_t lda, const float *X, int64_t ldx, float *C,
                        int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                        int ksplit, float *part, hipStream_t st) {
  return launch_main<false>(A, lda, X, ldx, C, ldc, M, N, K, alpha, beta, ksplit, part, st);
}

int launch_gemm_tn_main(const float *A, int64_t lda, const float *Y, int64_t ldy, float *C,
                        int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                        int ksplit, float *part, hipStream_t st) {
  return launch_main<true>(A, lda, Y, ldy, C, ldc, M, N, K, alpha, beta, ksplit, part, st);
}

void launch_gemm_nn(const float *A, int64_t lda, const float *X, int64_t ldx, float *C,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                    int ksplit, float *part, hipStream_t st) {
  const int nsp = launch_gemm_nn_main(A, lda, X, ldx, C, ldc, M, N, K, alpha, beta, ksplit,
                                      part, st);
  launch_gemm_finish(part, nsp, M, N, C, ldc, alpha, beta, st);
}

void launch_gemm_tn(const float *A, int64_t lda, const float *Y, int64_t ldy, float *C,
                    int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                    int ksplit, float *part, hipStream_t st) {
  const int nsp = launch_gemm_tn_main(A, lda, Y, ldy, C, ldc, M, N, K, alpha, beta, ksplit,
                                      part, st);
  launch_gemm_finish(part, nsp, M, N, C, ldc, alpha, beta, st);
}

}  // namespace farpca_int
