// A-passes of the precision form (A stored in BF16) on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation): the dense products A G_j and
// A^T Y_j of the power steps and block products (Algorithm 1/2), with the
// same NN / TN conventions as the FP32 kernels:
//
//   NN: C[M x N] = A[M x K] X[K x N]        (A row-major BF16, reduce along a row)
//   TN: C[M x N] = A^T Y, A is K x M        (A row-major BF16, reduce over rows)
//
// Exact skinny operand.  The FP32 skinny operand x is split into three BF16
// terms by rounding to nearest: hi = rn(x), mid = rn(x - hi), lo = x - hi -
// mid.  Each difference is exact in FP32 and x = hi + mid + lo exactly (lo has
// at most 8 significant bits while it is a normal number, |x| >= 2^-110, below
// which bits under 2^-126 are dropped), so three MFMAs
// per product reproduce the products A_ij x_j exactly (BF16 x BF16 products are
// exact in FP32) and only the FP32 accumulation rounds: the precision form
// computes what the FP32 path would compute on the BF16-rounded matrix.  At
// b = 64 the product is HBM-bound (2 flop per byte of A per output column
// pair); the tripled MFMA work fits under the HBM time.
//
// Skinny operand layout.  A pack kernel writes the skinny operand transposed
// (xt[c][k], K padded with zeros to whole groups of slices).  Per 32-deep K
// slice every thread of the workgroup loads 4 consecutive k of one column
// (16 bytes), splits them and stores the three BF16 planes into LDS
// (column-major, 40 BF16 = 80 bytes per column: 16-byte aligned reads).
//
// A workgroup has 8 waves; wave w owns the 64-row output tile t0 = 512 tile +
// 64 w and accumulates it in registers (16 accumulators of 16 x 16).  A is
// read straight into registers D slices ahead (a ring of D register slots,
// loop unrolled by D), the skinny slices D ahead as well, so that about D - 1
// slices of A (4 KB each per wave) are in flight at every point: HBM needs a
// few hundred KB in flight per CU.  One barrier per slice.
//
// K order inside a slice: MFMA lane (li = l % 16, lk = l / 16) holds 8 BF16 of
// its A row / column and 8 of its B column; element e of both is k = 8 lk + e.
//   NN: lane loads 16 bytes of A row t0 + 16 rt + li at k = 8 lk .. 8 lk + 7.
//   TN: lane loads 8 bytes (columns c0 + 4 li .. + 3) of the 8 A rows
//       8 lk .. 8 lk + 7 and regroups them per column t (byte permutes):
//       MFMA t's 16 output rows are columns c0 + 4 i + t (an interleaved
//       output tile, as in the FP32 TN kernel).
// Output D lane l element v = (row 4 (l/16) + v, column l % 16).
// Rows / columns outside the matrix are read at clamped addresses (finite
// values that meet zero skinny entries or feed outputs that are never stored).
//
// FP32 A.  The FP32 A-passes are bound by the FP32 matrix-core rate (157
// TFLOP/s: 2 m n b flop per 4 m n bytes needs 20 TB/s of A at b = 64), the
// BF16 matrix cores are 16 times faster: A is split in registers into three
// BF16 terms as well and six term products are formed, 6 x 2 m n b BF16 flop,
// well under the time it takes to stream A.  TN runs in the same kernel
// (F32 = true): each lane holds FP32 values (16 bytes per load) in the
// operand positions of the BF16 layout, 16 bytes (4 columns) of each of its 8
// rows, 256 contiguous bytes per row and instruction.  NN has a kernel of its
// own that stages A through LDS (gemm_f32s_nn_lds_kernel).
#include <map>
#include <mutex>
#include <tuple>

#include "internal.h"

namespace farpca_int {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kB16Waves = 8;
constexpr int kB16Threads = 64 * kB16Waves;
constexpr int kB16Rows = 64 * kB16Waves;      // output rows per workgroup
constexpr int kKGroup = 192;                  // K granularity of splits and padding

// Per layout: SL K rows per slice (32 per MFMA step), RING slices in the
// register ring, NBUF staged skinny slices in LDS.  NN slices are 64 deep so
// that a lane's two 16-byte loads of a row are back-to-back halves of one
// 128-byte line (64-byte row pieces one slice apart stream at a much lower HBM
// rate); TN rows are read as 128-byte runs already.
template <bool TN, bool F32> struct B16Cfg;
template <> struct B16Cfg<true, false> {
  static constexpr int SL = 32, RING = 6, NBUF = 2, AV = 4;
};
template <> struct B16Cfg<false, false> {
  static constexpr int SL = 64, RING = 3, NBUF = 3, AV = 8;
};
// FP32 A (TN): a slot holds 8 float4 per lane (4 columns of 8 rows), so the
// ring is shallower (two slots: the per-slice accumulators of mma_slice_f32
// take the registers of a third, at the same measured speed); 32-deep slices.
template <> struct B16Cfg<true, true> {
  static constexpr int SL = 32, RING = 2, NBUF = 2, AV = 8;
};
template <bool TN, bool F32> struct B16Lds {
  static constexpr int CS = B16Cfg<TN, F32>::SL + 8;   // BF16 per staged column (16-byte aligned)
  static constexpr int PLANE = kBld * CS;               // BF16 per split plane
  static constexpr int STAGE = 3 * PLANE;               // BF16 per staged slice
  static constexpr int XL = B16Cfg<TN, F32>::SL / 32;   // float4 skinny pieces per thread per slice
};
template <bool TN, bool F32> constexpr int kGroup = B16Cfg<TN, F32>::SL * B16Cfg<TN, F32>::RING;
static_assert(kGroup<true, false> == kKGroup && kGroup<false, false> == kKGroup, "BF16 groups");
static_assert(kKGroup % kGroup<true, true> == 0, "FP32 groups divide the split granularity");
static_assert(kB16Threads == kBld * 8, "eight column pieces per skinny column");
static_assert(B16Cfg<true, false>::RING % B16Cfg<true, false>::NBUF == 0 &&
                  B16Cfg<false, false>::RING % B16Cfg<false, false>::NBUF == 0 &&
                  B16Cfg<true, true>::RING % B16Cfg<true, true>::NBUF == 0,
              "static LDS buffer of every unrolled step");

__device__ __forceinline__ floatx4 mfma_bf16(u32x4 a, u32x4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ __forceinline__ int64_t b16_clamp(int64_t v, int64_t hi) { return v < hi ? v : hi; }

// Logical workgroup id (consecutive ids, i.e. one K split, on one XCD).
__device__ __forceinline__ int64_t b16_xcd_remap(int64_t g, int64_t T) {
  const int64_t T8 = T & ~int64_t(7);
  if (g >= T8) return g;
  return (g & 7) * (T8 >> 3) + (g >> 3);
}

// ------------------------------------------------------------------ pack
// xt[c * kp + k] = X[k][c] for k < K, c < N; zero elsewhere (k < kp, c < 64).
__global__ __launch_bounds__(256) void bf16_pack_kernel(const float *__restrict__ X, int64_t ldx,
                                                        int64_t K, int64_t N, int64_t kp,
                                                        float *__restrict__ xt) {
  __shared__ float t[64][65];
  const int64_t k0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int64_t k = k0 + r;
    t[c][r] = (k < K && c < N) ? X[k * ldx + c] : 0.0f;
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int c = e >> 6, r = e & 63;
    const int64_t k = k0 + r;
    if (k < kp) xt[c * kp + k] = t[c][r];
  }
}

// ---------------------------------------------------------- A slot loads
// NN: v[2 rt + ks] = row group rt, MFMA step ks; TN: rows (2 j, 2 j + 1) in v[j].
template <bool TN, bool F32> struct ASlot { u32x4 v[B16Cfg<TN, F32>::AV]; };
template <bool TN> struct ASlot<TN, true> { float4 v[B16Cfg<TN, true>::AV]; };

// AVEC, NN: rows hold whole groups of 8 up to k8 = K rounded up to 8 (K % 8
// == 0, or lda >= k8): a group is read at its start clamped to k8 - 8, and
// when K % 8 != 0 its elements at k >= K are set to zero (the row padding may
// hold anything).  AVEC, TN: columns are read in groups of 4 clamped to
// mclamp - 4 (mclamp = M rounded up to 4 when lda allows; the columns past M
// only feed outputs that are never stored).
template <bool TN, bool AVEC>
__device__ __forceinline__ void load_slot(const uint16_t *A, int64_t lda, int64_t M,
                                          int64_t K, int64_t t0, int li, int lk, int64_t k0,
                                          ASlot<TN, false> &s, int64_t mclamp) {
  if constexpr (!TN) {
    const int64_t k8 = (K + 7) & ~int64_t(7);
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int64_t row = b16_clamp(t0 + 16 * rt + li, M - 1);
      const uint16_t *p = A + row * lda;
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const int64_t kk = k0 + 32 * ks + 8 * lk;
        if (AVEC) {
          const int64_t g = b16_clamp(kk, k8 - 8);
          u32x4 v = *reinterpret_cast<const u32x4 *>(p + g);
          if ((K & 7) != 0 && g + 8 > K) {
            const int64_t nv = K - g;            // 1 .. 7 valid elements
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const uint32_t lo = (2 * q < nv) ? 0x0000FFFFu : 0u;
              const uint32_t hi = (2 * q + 1 < nv) ? 0xFFFF0000u : 0u;
              w[q] &= lo | hi;
            }
            v = u32x4{w[0], w[1], w[2], w[3]};
          }
          s.v[2 * rt + ks] = v;
        } else {
          uint32_t h[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) h[e] = p[b16_clamp(kk + e, K - 1)];
          s.v[2 * rt + ks] = u32x4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16),
                                   h[6] | (h[7] << 16)};
        }
      }
    }
  } else {
    const int64_t c = t0 + 4 * li;
    // rows k0 + 8 lk + q: pointer of the lane's first row plus q lda (the
    // slice base k0 lda is uniform); rows past K read row K - 1
    const int64_t cc = AVEC ? b16_clamp(c, mclamp - 4) : c;
    const uint16_t *pc = A + cc;
    const uint16_t *plast = pc + (K - 1) * lda;
    const uint16_t *p0 = pc + k0 * lda + 8 * lk * lda;
    const int64_t r0 = k0 + 8 * lk;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      uint32_t w[4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = 2 * j + h;
        const uint16_t *p = (r0 + q < K) ? p0 + q * lda : plast;
        if (AVEC) {
          // columns c .. c + 3 are inside the row (or its padding) or the whole group is clamped
          const uint2 u = *reinterpret_cast<const uint2 *>(p);
          w[2 * h] = u.x;
          w[2 * h + 1] = u.y;
        } else {
          uint32_t v[4];
#pragma unroll
          for (int t = 0; t < 4; ++t) v[t] = p[b16_clamp(c + t, M - 1) - c];
          w[2 * h] = v[0] | (v[1] << 16);
          w[2 * h + 1] = v[2] | (v[3] << 16);
        }
      }
      s.v[j] = u32x4{w[0], w[1], w[2], w[3]};
    }
  }
}

// TN: the MFMA operand of column t (0..3) of the lane's 4 columns: element e =
// row 8 lk + e.  v[j] holds row 2 j in (x, y) and row 2 j + 1 in (z, w), each
// row as (columns 0,1), (columns 2,3).
__device__ __forceinline__ u32x4 tn_operand(const ASlot<true, false> &s, int t) {
  uint32_t d[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t r0 = (t < 2) ? s.v[j].x : s.v[j].y;   // row 2 j
    const uint32_t r1 = (t < 2) ? s.v[j].z : s.v[j].w;   // row 2 j + 1
    d[j] = (t & 1) ? ((r0 >> 16) | (r1 & 0xFFFF0000u)) : ((r0 & 0xFFFFu) | (r1 << 16));
  }
  return u32x4{d[0], d[1], d[2], d[3]};
}


typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));

// Two FP32 values rounded to nearest BF16 (v_cvt_pk_bf16_f32), the first in the
// low half.
__device__ __forceinline__ uint32_t rn_pair(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((floatx2){a, b}, bf16x2));
}

// Exact split of two FP32 values into three BF16 terms each, packed in pairs:
// hi = rn(v), mid = rn(v - hi), lo = v - hi - mid.  Both differences are exact
// in FP32 (|v - hi| <= 2^-8 |v| on the FP32 grid of v), and lo has at most 8
// significant bits, so v = hi + mid + lo exactly while lo is a normal number
// (|v| >= 2^-110; below that, bits under 2^-126 are dropped); |mid| <= 2^-8
// |v|, |lo| <= 2^-16 |v|, and the residuals take either sign.
__device__ __forceinline__ void split_pair(float a0, float a1, uint32_t &h, uint32_t &m, uint32_t &l) {
  h = rn_pair(a0, a1);
  const float r0 = a0 - __uint_as_float(h << 16);             // exact
  const float r1 = a1 - __uint_as_float(h & 0xFFFF0000u);
  m = rn_pair(r0, r1);
  const float s0 = r0 - __uint_as_float(m << 16);             // exact, <= 8 bits
  const float s1 = r1 - __uint_as_float(m & 0xFFFF0000u);
  l = rn_pair(s0, s1);                                        // exact
}

// The thread's 4 XL skinny values (k = 4 XL kq .. + 4 XL - 1 of column sc)
// into the three BF16 planes of the staged slice.
template <bool TN, bool F32>
__device__ __forceinline__ void stage_skinny(uint16_t *xs, int sc, int kq,
                                             const float4 (&x)[B16Lds<TN, F32>::XL]) {
  using Lds = B16Lds<TN, F32>;
  uint16_t *col = xs + sc * Lds::CS;
#pragma unroll
  for (int g = 0; g < Lds::XL; ++g) {
    const int pos = 4 * (Lds::XL * kq + g);
    uint32_t h0, m0, l0, h1, m1, l1;
    split_pair(x[g].x, x[g].y, h0, m0, l0);
    split_pair(x[g].z, x[g].w, h1, m1, l1);
    *reinterpret_cast<uint2 *>(col + pos) = make_uint2(h0, h1);
    *reinterpret_cast<uint2 *>(col + pos + Lds::PLANE) = make_uint2(m0, m1);
    *reinterpret_cast<uint2 *>(col + pos + 2 * Lds::PLANE) = make_uint2(l0, l1);
  }
}

template <bool TN>
__device__ __forceinline__ void mma_slice_bf16(floatx4 (&acc)[16], const ASlot<TN, false> &s,
                                               const uint16_t *xs, int li, int lk) {
  using Lds = B16Lds<TN, false>;
  constexpr int KS = B16Cfg<TN, false>::SL / 32;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    u32x4 a[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      if constexpr (TN) a[x] = tn_operand(s, x);
      else a[x] = s.v[2 * x + ks];
    }
    const uint16_t *xb = xs + li * Lds::CS + 32 * ks + 8 * lk;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const u32x4 bop = *reinterpret_cast<const u32x4 *>(xb + p * Lds::PLANE + 16 * ct * Lds::CS);
#pragma unroll
        for (int x = 0; x < 4; ++x) acc[x * 4 + ct] = mfma_bf16(a[x], bop, acc[x * 4 + ct]);
      }
    }
  }
}

// ------------------------------------------------------- FP32 A operand
// FP32 A, TN: v[q] = row k0 + 8 lk + q, columns t0 + 4 li .. + 3 (AVEC: the
// group clamped to mclamp - 4 as for BF16); rows past K read row K - 1 (they
// meet zero skinny rows), clamped columns feed outputs that are never stored.
template <bool AVEC>
__device__ __forceinline__ void load_slot_f32(const float *A, int64_t lda, int64_t M, int64_t K,
                                              int64_t t0, int li, int lk, int64_t k0,
                                              ASlot<true, true> &s, int64_t mclamp) {
  const int64_t c = t0 + 4 * li;
  const int64_t cc = AVEC ? b16_clamp(c, mclamp - 4) : c;
  const float *pc = A + cc;
  const float *plast = pc + (K - 1) * lda;
  const float *p0 = pc + k0 * lda + 8 * lk * lda;
  const int64_t r0 = k0 + 8 * lk;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float *p = (r0 + q < K) ? p0 + q * lda : plast;
    if (AVEC) {
      s.v[q] = *reinterpret_cast<const float4 *>(p);
    } else {
      s.v[q] = make_float4(p[b16_clamp(c, M - 1) - c], p[b16_clamp(c + 1, M - 1) - c],
                           p[b16_clamp(c + 2, M - 1) - c], p[b16_clamp(c + 3, M - 1) - c]);
    }
  }
}

// The MFMA operand of 8 FP32 values of A as three BF16 planes (split_pair).
__device__ __forceinline__ void split8(const float (&e)[8], u32x4 &hi, u32x4 &mid, u32x4 &lo) {
  uint32_t h[4], m[4], l[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) split_pair(e[2 * j], e[2 * j + 1], h[j], m[j], l[j]);
  hi = u32x4{h[0], h[1], h[2], h[3]};
  mid = u32x4{m[0], m[1], m[2], m[3]};
  lo = u32x4{l[0], l[1], l[2], l[3]};
}

// One 32-deep slice with FP32 A: both operands split in three, six of the nine
// products (hi hi, hi mid, mid hi, mid mid, hi lo, lo hi).  The three left out
// (mid lo, lo mid, lo lo) are below 2^-23 of |a x| together (|mid| <= 2^-8,
// |lo| <= 2^-16 of either operand) and of either sign: about one FP32
// rounding of the product.
// The six term products of one 16-row group of A (planes ah, am, al) with the
// four 16-column tiles of the staged skinny planes b, accumulated in acc4[ct]
// (all column tiles of a product before the next product).
__device__ __forceinline__ void mma_split6(floatx4 *acc4, const u32x4 &ah, const u32x4 &am,
                                           const u32x4 &al, const u32x4 (&b)[3][4]) {
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc4[ct] = mfma_bf16(ah, b[0][ct], acc4[ct]);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc4[ct] = mfma_bf16(ah, b[1][ct], acc4[ct]);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc4[ct] = mfma_bf16(am, b[0][ct], acc4[ct]);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc4[ct] = mfma_bf16(am, b[1][ct], acc4[ct]);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc4[ct] = mfma_bf16(ah, b[2][ct], acc4[ct]);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc4[ct] = mfma_bf16(al, b[0][ct], acc4[ct]);
}

// The three skinny planes of MFMA step ks for lane (li, lk): b[p][ct].
template <typename Lds>
__device__ __forceinline__ void load_b_planes(const uint16_t *xs, int li, int lk, int ks,
                                              u32x4 (&b)[3][4]) {
  const uint16_t *xb = xs + li * Lds::CS + 32 * ks + 8 * lk;
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      b[p][ct] = *reinterpret_cast<const u32x4 *>(xb + p * Lds::PLANE + 16 * ct * Lds::CS);
}

// One 32-deep TN slice with FP32 A: column t of the lane's 4 (output rows
// t0 + 4 li + t) is MFMA row group t.  The slice's six term products start
// from zero and their sum is added to the running accumulator by the vector
// unit (FP32, round to nearest): accumulated inside the matrix cores over the
// whole K, the products of C_j^T = A^T Q_j left a bias in the indicator of the
// order of 1e-7 ||A||^2 (sums of squares of many columns), which this removes.
__device__ __forceinline__ void mma_slice_f32(floatx4 (&acc)[16], const ASlot<true, true> &s,
                                              const uint16_t *xs, int li, int lk) {
  static_assert(B16Cfg<true, true>::SL == 32, "one MFMA step per slice");
  u32x4 b[3][4];
  load_b_planes<B16Lds<true, true>>(xs, li, lk, 0, b);
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    float e[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float4 &r = s.v[q];
      e[q] = x == 0 ? r.x : (x == 1 ? r.y : (x == 2 ? r.z : r.w));
    }
    u32x4 ah, am, al;
    split8(e, ah, am, al);
    floatx4 t[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) t[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
    mma_split6(t, ah, am, al, b);
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[4 * x + ct] += t[ct];
  }
}

// F32: A holds FP32 values (split in registers), else BF16 bit patterns.
template <bool TN, bool AVEC, bool F32>
__global__ __launch_bounds__(kB16Threads) void gemm_bf16_kernel(
    const void *Av, int64_t lda, const float *xt, int64_t kp, float *__restrict__ C, int64_t ldc,
    int64_t M, int64_t N, int64_t K, int64_t kps, int64_t tiles, int64_t total, float alpha,
    float beta, float *__restrict__ part, int64_t mclamp) {
  using Cfg = B16Cfg<TN, F32>;
  using Lds = B16Lds<TN, F32>;
  constexpr int G = kGroup<TN, F32>;
  constexpr int SL = Cfg::SL, RING = Cfg::RING, NBUF = Cfg::NBUF, XL = Lds::XL;
  __shared__ __attribute__((aligned(16))) uint16_t xs[NBUF][Lds::STAGE];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t L = b16_xcd_remap(blockIdx.x, total);
  const int64_t tile = L % tiles, split = L / tiles;
  static_assert(TN || !F32, "FP32 A, NN: gemm_f32s_nn_lds_kernel");
  const int64_t t0 = tile * kB16Rows + 64 * wave;
  const int64_t kb = split * kps;
  const int64_t ke = (kb + kps < K) ? kb + kps : K;
  // slices of this split, a multiple of RING (kps is a multiple of kKGroup, a
  // multiple of G = SL RING; slices past K meet zero skinny rows)
  const int64_t nsl = ((ke - kb + G - 1) / G) * RING;
  const int sc = tid >> 3, kq = tid & 7;
  const float *xsrc = xt + sc * kp + kb + 4 * XL * kq;

  floatx4 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};

  ASlot<TN, F32> ar[RING];
  float4 xr[RING][XL];
  // Every slice's loads are issued in one fixed order (skinny pieces, then A),
  // in the prologue as in the loop: the wait counts the compiler derives from
  // that order keep RING - 1 slices in flight (a different prologue order
  // makes it wait for nearly everything at the loop head).
  auto issue = [&](int64_t s, int slot) {
    const int64_t sl = s < nsl ? s : nsl - 1;      // clamped: in bounds, never used
#pragma unroll
    for (int g = 0; g < XL; ++g) xr[slot][g] = *reinterpret_cast<const float4 *>(xsrc + sl * SL + 4 * g);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (F32)
      load_slot_f32<AVEC>(static_cast<const float *>(Av), lda, M, K, t0, li, lk, kb + sl * SL,
                              ar[slot], mclamp);
    else
      load_slot<TN, AVEC>(static_cast<const uint16_t *>(Av), lda, M, K, t0, li, lk, kb + sl * SL,
                          ar[slot], mclamp);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  };
#pragma unroll
  for (int d = 0; d < RING; ++d) issue(d, d);
  stage_skinny<TN, F32>(xs[0], sc, kq, xr[0]);

  for (int64_t s0 = 0; s0 < nsl; s0 += RING) {
#pragma unroll
    for (int d = 0; d < RING; ++d) {
      // RING is a multiple of NBUF: slice s0 + d lives in buffer d % NBUF
      const int buf = d % NBUF;
      __syncthreads();                 // slice s0 + d staged; slice s0 + d - 1 consumed
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (F32) mma_slice_f32(acc, ar[d], xs[buf], li, lk);
      else mma_slice_bf16<TN>(acc, ar[d], xs[buf], li, lk);
      __builtin_amdgcn_sched_barrier(0);
      stage_skinny<TN, F32>(xs[(d + 1) % NBUF], sc, kq, xr[(d + 1) % RING]);
      issue(s0 + d + RING, d);
      __builtin_amdgcn_sched_barrier(0);
    }
  }

  float *dst = part ? part + split * M * kBld : C;
  const int64_t ld = part ? kBld : ldc;
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
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

// ------------------------------------------- FP32 A, NN, A staged in LDS
// A G with FP32 A.  Read straight into the MFMA operand layout, a load
// instruction covers 16 rows x 64 bytes and the pass streams A at about 3 TB/s
// whatever the arithmetic; here each wave reads the 64-deep slice of its own
// 16 rows as 4 rows x 256 contiguous bytes per instruction (16 lanes per row),
// kNlRing slices ahead in registers, stores it into its own part of LDS (row
// stride 68 floats: the 16-byte stores of a row and the 16-byte operand reads
// of 8 consecutive rows are bank-conflict free) and reads its MFMA operands
// back from there.  No other wave touches those rows, and a wave's LDS
// accesses run in order, so the A tile needs no barrier.  The skinny slice
// (split into its three BF16 planes once per workgroup, in its natural k
// order) is shared by the 16 waves and double-buffered: one barrier per slice,
// after which the next slice's A loads are already in flight and its skinny
// planes are staged once the MFMAs of this one are issued.  The skinny planes
// are read one at a time (hi: three products, mid: two, lo: one), so that a
// wave fits in 128 registers and four waves share a SIMD.  LDS: 16 x 16 x 68
// floats (68 KB) of A and 2 x 27 KB of skinny planes.
constexpr int kNlRows = 256;                 // output rows per workgroup
constexpr int kNlSl = 64;                    // k per slice
constexpr int kNlLd = kNlSl + 4;             // floats per LDS row of the tile
constexpr int kNlRing = 2;                   // slices in flight in registers
static_assert(kKGroup % kNlSl == 0, "slices divide the split granularity");

constexpr int kNlWaves = 16;
constexpr int kNlThreads = 64 * kNlWaves;

template <bool AVEC>
__global__ __launch_bounds__(kNlThreads) void gemm_f32s_nn_lds_kernel(
    const float *__restrict__ A, int64_t lda, const float *xt, int64_t kp, float *__restrict__ C,
    int64_t ldc, int64_t M, int64_t N, int64_t K, int64_t kps, int64_t tiles, int64_t total,
    float alpha, float beta, float *__restrict__ part) {
  using Lds = B16Lds<false, false>;                 // 64-deep skinny slices, natural k order
  static_assert(B16Cfg<false, false>::SL == kNlSl, "skinny slice layout");
  // A: each wave stages its own 16 rows (no other wave reads them); the
  // skinny planes are shared and double-buffered
  __shared__ __attribute__((aligned(16))) float al[kNlWaves * 16 * kNlLd];
  __shared__ __attribute__((aligned(16))) uint16_t xs[2 * Lds::STAGE];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t L = b16_xcd_remap(blockIdx.x, total);
  const int64_t tile = L % tiles, split = L / tiles;
  const int64_t r0 = tile * kNlRows;
  const int64_t kb = split * kps;
  const int64_t ke = (kb + kps < K) ? kb + kps : K;
  const int64_t nsl = (ke - kb + kNlSl - 1) / kNlSl;
  const int sc = tid >> 4, kq = tid & 15;
  const float *xsrc = xt + sc * kp + kb + 4 * kq;
  const int wrow = 16 * wave;
  float *aw = al + wrow * kNlLd;                    // this wave's 16 rows

  floatx4 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};

  constexpr int R = kNlRing;
  float4 ar[R][4];
  float4 xr[R];
  // wave w reads rows wrow + 4 q + lane / 16, 16 lanes per row (256 bytes)
  auto issue = [&](int64_t s, int slot) {
    const int64_t sl = s < nsl ? s : nsl - 1;      // clamped: in bounds, never used
    xr[slot] = *reinterpret_cast<const float4 *>(xsrc + sl * kNlSl);
    const int64_t k0 = kb + sl * kNlSl;
    const int64_t kk = k0 + 4 * li;
    const int64_t k4 = (K + 3) & ~int64_t(3);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = b16_clamp(r0 + wrow + 4 * q + lk, M - 1);
      const float *p = A + row * lda;
      if (AVEC) {
        const int64_t g = b16_clamp(kk, k4 - 4);
        float4 x = *reinterpret_cast<const float4 *>(p + g);
        if ((K & 3) != 0 && g + 4 > K) {
          const int64_t nv = K - g;                // 1 .. 3 valid elements
          x.y = nv > 1 ? x.y : 0.0f;
          x.z = nv > 2 ? x.z : 0.0f;
          x.w = 0.0f;
        }
        ar[slot][q] = x;
      } else {
        ar[slot][q] = make_float4(p[b16_clamp(kk, K - 1)], p[b16_clamp(kk + 1, K - 1)],
                                  p[b16_clamp(kk + 2, K - 1)], p[b16_clamp(kk + 3, K - 1)]);
      }
    }
  };
  auto stage_x = [&](int slot, int buf) {
    uint32_t h0, m0, l0, h1, m1, l1;
    split_pair(xr[slot].x, xr[slot].y, h0, m0, l0);
    split_pair(xr[slot].z, xr[slot].w, h1, m1, l1);
    uint16_t *col = xs + buf * Lds::STAGE + sc * Lds::CS + 4 * kq;
    *reinterpret_cast<uint2 *>(col) = make_uint2(h0, h1);
    *reinterpret_cast<uint2 *>(col + Lds::PLANE) = make_uint2(m0, m1);
    *reinterpret_cast<uint2 *>(col + 2 * Lds::PLANE) = make_uint2(l0, l1);
  };
#pragma unroll
  for (int d = 0; d < R; ++d) issue(d, d);
  stage_x(0, 0);
  for (int64_t s0 = 0; s0 < nsl; s0 += R) {
#pragma unroll
    for (int d = 0; d < R; ++d) {
      const int64_t s = s0 + d;
      if (s >= nsl) break;                         // uniform
      const int buf = (int)(s & 1);
      // this wave's rows of slice s; its reads of slice s - 1 were issued
      // first and a wave's LDS accesses run in order
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int q = 0; q < 4; ++q)
        *reinterpret_cast<float4 *>(aw + (4 * q + lk) * kNlLd + 4 * li) = ar[d][q];
      __builtin_amdgcn_wave_barrier();
      issue(s + R, d);
      // skinny slice s staged by every wave; slice s - 1's buffer free
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        const float *ap = aw + li * kNlLd + 32 * ks + 8 * lk;
        const float4 u = *reinterpret_cast<const float4 *>(ap);
        const float4 w = *reinterpret_cast<const float4 *>(ap + 4);
        const float e[8] = {u.x, u.y, u.z, u.w, w.x, w.y, w.z, w.w};
        u32x4 ah, am, alo;
        split8(e, ah, am, alo);
        const uint16_t *xb = xs + buf * Lds::STAGE + li * Lds::CS + 32 * ks + 8 * lk;
        u32x4 b[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) b[ct] = *reinterpret_cast<const u32x4 *>(xb + 16 * ct * Lds::CS);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma_bf16(ah, b[ct], acc[ct]);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma_bf16(am, b[ct], acc[ct]);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma_bf16(alo, b[ct], acc[ct]);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) b[ct] = *reinterpret_cast<const u32x4 *>(xb + Lds::PLANE + 16 * ct * Lds::CS);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma_bf16(ah, b[ct], acc[ct]);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma_bf16(am, b[ct], acc[ct]);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) b[ct] = *reinterpret_cast<const u32x4 *>(xb + 2 * Lds::PLANE + 16 * ct * Lds::CS);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma_bf16(ah, b[ct], acc[ct]);
      }
      if (s + 1 < nsl) stage_x((d + 1) % R, buf ^ 1);
    }
  }

  float *dst = part ? part + split * M * kBld : C;
  const int64_t ld = part ? kBld : ldc;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + wrow + 4 * lk + v;
      const int64_t col = 16 * ct + li;
      if (row < M && col < N) {
        float r = acc[ct][v];
        if (!part) {
          r *= alpha;
          if (beta != 0.0f) r += beta * dst[row * ld + col];
        }
        dst[row * ld + col] = r;
      }
    }
}

// ------------------------------------------------------------------ host
static int64_t bf16_slots(int is_tn, bool f32) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, int>, int64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_tuple(dev, is_tn, f32 ? 1 : 0);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  const void *fn =
      f32 ? (is_tn ? reinterpret_cast<const void *>(&gemm_bf16_kernel<true, true, true>)
                   : reinterpret_cast<const void *>(&gemm_f32s_nn_lds_kernel<true>))
          : (is_tn ? reinterpret_cast<const void *>(&gemm_bf16_kernel<true, true, false>)
                   : reinterpret_cast<const void *>(&gemm_bf16_kernel<false, true, false>));
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, (f32 && !is_tn) ? kNlThreads : kB16Threads,
                                                   0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int64_t slots = (int64_t)cus * per_cu;
  cache[key] = slots;
  return slots;
}

int64_t bf16_padded_k(int64_t K) { return (K + kKGroup - 1) / kKGroup * kKGroup; }

// K splits: as for the FP32 kernels (rounds of resident workgroups x split
// length, partial tiles cheap next to A), splits in whole groups of kKGroup
// (so a short K still spreads over several workgroups per 512-row tile).
static int choose_ksplit(int64_t M, int64_t K, int is_tn, int64_t max_split, bool f32) {
  if (M < 1 || K < 1) return 1;
  const int64_t rows = (f32 && !is_tn) ? kNlRows : kB16Rows;
  const int64_t tiles = (M + rows - 1) / rows;
  const int64_t slots = bf16_slots(is_tn, f32);
  int64_t smax = K / kKGroup;
  if (smax > max_split) smax = max_split;
  if (smax > 64) smax = 64;
  int best = 1;
  double best_cost = 0.0;
  for (int64_t sp = 1; sp <= (smax < 1 ? 1 : smax); ++sp) {
    const int64_t rounds = (tiles * sp + slots - 1) / slots;
    const double cost = (double)rounds / (double)sp * (1.0 + 128.0 * (double)sp / (double)K);
    if (sp == 1 || cost < best_cost * (1.0 - 1e-9)) {
      best = (int)sp;
      best_cost = cost;
    }
  }
  return best;
}

int gemm_bf16_choose_ksplit(int64_t M, int64_t K, int is_tn, int64_t max_split) {
  return choose_ksplit(M, K, is_tn, max_split, false);
}

int gemm_f32s_choose_ksplit(int64_t M, int64_t K, int is_tn, int64_t max_split) {
  return choose_ksplit(M, K, is_tn, max_split, true);
}

size_t bf16_pack_bytes(int64_t K) { return (size_t)bf16_padded_k(K) * kBld * sizeof(float); }

template <bool TN, bool F32>
static int launch_bf16(const void *A, int64_t lda, const float *X, int64_t ldx, float *C,
                       int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                       int ksplit, float *part, float *xt, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return 1;
  if (ksplit < 1) ksplit = 1;
  const int64_t kp = bf16_padded_k(K);
  hipLaunchKernelGGL(bf16_pack_kernel, dim3((unsigned)((kp + 63) / 64)), dim3(256), 0, st, X, ldx,
                     K, N, kp, xt);
  int64_t kps = (K + ksplit - 1) / ksplit;
  kps = (kps + kKGroup - 1) / kKGroup * kKGroup;
  const int nsp = (int)((K + kps - 1) / kps);
  float *p = (nsp > 1) ? part : nullptr;
  constexpr int64_t rows = (F32 && !TN) ? kNlRows : kB16Rows;
  const int64_t tiles = (M + rows - 1) / rows;
  const int64_t total = tiles * nsp;
  const uintptr_t ad = reinterpret_cast<uintptr_t>(A);
  // vector loads: aligned rows whose groups of 4 columns (TN: 8 bytes BF16,
  // 16 bytes FP32) / of 8 (BF16) or 4 (FP32) k (NN) stay inside the row or its
  // padding up to lda
  const int64_t m4 = (M + 3) / 4 * 4, k8 = (K + 7) / 8 * 8, k4 = (K + 3) / 4 * 4;
  bool avec;
  if (F32)
    avec = TN ? (M >= 4 && lda % 4 == 0 && (ad & 15) == 0 && (M % 4 == 0 || lda >= m4))
              : (K >= 4 && lda % 4 == 0 && (ad & 15) == 0 && (K % 4 == 0 || lda >= k4));
  else
    avec = TN ? (M >= 4 && lda % 4 == 0 && (ad & 7) == 0 && (M % 4 == 0 || lda >= m4))
              : (K >= 8 && lda % 8 == 0 && (ad & 15) == 0 && (K % 8 == 0 || lda >= k8));
  const int64_t mclamp = (TN && M % 4 != 0) ? m4 : M;
  dim3 grid((unsigned)total), blk(kB16Threads);
  if constexpr (F32 && !TN) {
    blk = dim3(kNlThreads);
    const float *Af = static_cast<const float *>(A);
    if (avec)
      hipLaunchKernelGGL((gemm_f32s_nn_lds_kernel<true>), grid, blk, 0, st, Af, lda, xt, kp, C, ldc,
                         M, N, K, kps, tiles, total, alpha, beta, p);
    else
      hipLaunchKernelGGL((gemm_f32s_nn_lds_kernel<false>), grid, blk, 0, st, Af, lda, xt, kp, C, ldc,
                         M, N, K, kps, tiles, total, alpha, beta, p);
  } else {
    if (avec)
      hipLaunchKernelGGL((gemm_bf16_kernel<TN, true, F32>), grid, blk, 0, st, A, lda, xt, kp, C, ldc,
                         M, N, K, kps, tiles, total, alpha, beta, p, mclamp);
    else
      hipLaunchKernelGGL((gemm_bf16_kernel<TN, false, F32>), grid, blk, 0, st, A, lda, xt, kp, C, ldc,
                         M, N, K, kps, tiles, total, alpha, beta, p, mclamp);
  }
  return nsp;
}

int launch_gemm_bf16_nn_main(const uint16_t *A, int64_t lda, const float *X, int64_t ldx, float *C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                             int ksplit, float *part, float *xt, hipStream_t st) {
  return launch_bf16<false, false>(A, lda, X, ldx, C, ldc, M, N, K, alpha, beta, ksplit, part, xt, st);
}

int launch_gemm_bf16_tn_main(const uint16_t *A, int64_t lda, const float *Y, int64_t ldy, float *C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                             int ksplit, float *part, float *xt, hipStream_t st) {
  return launch_bf16<true, false>(A, lda, Y, ldy, C, ldc, M, N, K, alpha, beta, ksplit, part, xt, st);
}

int launch_gemm_f32s_nn_main(const float *A, int64_t lda, const float *X, int64_t ldx, float *C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                             int ksplit, float *part, float *xt, hipStream_t st) {
  return launch_bf16<false, true>(A, lda, X, ldx, C, ldc, M, N, K, alpha, beta, ksplit, part, xt, st);
}

int launch_gemm_f32s_tn_main(const float *A, int64_t lda, const float *Y, int64_t ldy, float *C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                             int ksplit, float *part, float *xt, hipStream_t st) {
  return launch_bf16<true, true>(A, lda, Y, ldy, C, ldc, M, N, K, alpha, beta, ksplit, part, xt, st);
}

}  // namespace farpca_int
