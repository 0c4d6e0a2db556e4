// A-passes of the precision form (A stored in BF16) on the BF16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation): the dense products A G_j and
// A^T Y_j of the power steps and block products (Algorithm 1/2), with the
// same NN / TN conventions as the FP32 kernels:
//
//   NN: C[M x N] = A[M x K] X[K x N]        (A row-major BF16, reduce along a row)
//   TN: C[M x N] = A^T Y, A is K x M        (A row-major BF16, reduce over rows)
//
// Exact skinny operand.  The FP32 skinny operand x is split into three BF16
// terms by truncation: hi = x with the low 16 bits cleared, mid = (x - hi)
// truncated the same way, lo = x - hi - mid.  Each difference is exact in FP32
// and x = hi + mid + lo exactly (24 significand bits = 3 x 8; while lo is a
// normal number, |x| >= 2^-110, below which bits under 2^-126 are dropped), so three MFMAs
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
template <bool TN> struct B16Cfg;
template <> struct B16Cfg<true> {
  static constexpr int SL = 32, RING = 6, NBUF = 2, AV = 4;
};
template <> struct B16Cfg<false> {
  static constexpr int SL = 64, RING = 3, NBUF = 3, AV = 8;
};
template <bool TN> struct B16Lds {
  static constexpr int CS = B16Cfg<TN>::SL + 8;   // BF16 per staged column (16-byte aligned)
  static constexpr int PLANE = kBld * CS;          // BF16 per split plane
  static constexpr int STAGE = 3 * PLANE;          // BF16 per staged slice
  static constexpr int XL = B16Cfg<TN>::SL / 32;   // float4 skinny pieces per thread per slice
};
static_assert(B16Cfg<true>::SL * B16Cfg<true>::RING == kKGroup, "TN group");
static_assert(B16Cfg<false>::SL * B16Cfg<false>::RING == kKGroup, "NN group");
static_assert(kB16Threads == kBld * 8, "eight column pieces per skinny column");
static_assert(B16Cfg<true>::RING % B16Cfg<true>::NBUF == 0 && B16Cfg<false>::RING % B16Cfg<false>::NBUF == 0,
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
template <bool TN> struct ASlot { u32x4 v[B16Cfg<TN>::AV]; };

// AVEC, NN: rows hold whole groups of 8 up to k8 = K rounded up to 8 (K % 8
// == 0, or lda >= k8): a group is read at its start clamped to k8 - 8, and
// when K % 8 != 0 its elements at k >= K are set to zero (the row padding may
// hold anything).  AVEC, TN: columns are read in groups of 4 clamped to
// mclamp - 4 (mclamp = M rounded up to 4 when lda allows; the columns past M
// only feed outputs that are never stored).
template <bool TN, bool AVEC>
__device__ __forceinline__ void load_slot(const uint16_t *A, int64_t lda, int64_t M,
                                          int64_t K, int64_t t0, int li, int lk, int64_t k0,
                                          ASlot<TN> &s, int64_t mclamp) {
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
__device__ __forceinline__ u32x4 tn_operand(const ASlot<true> &s, int t) {
  uint32_t d[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t r0 = (t < 2) ? s.v[j].x : s.v[j].y;   // row 2 j
    const uint32_t r1 = (t < 2) ? s.v[j].z : s.v[j].w;   // row 2 j + 1
    d[j] = (t & 1) ? ((r0 >> 16) | (r1 & 0xFFFF0000u)) : ((r0 & 0xFFFFu) | (r1 << 16));
  }
  return u32x4{d[0], d[1], d[2], d[3]};
}

// Split the thread's 4 XL FP32 skinny values (k = 4 XL kq .. + 4 XL - 1 of
// column sc) into the three BF16 planes of the staged slice.
__device__ __forceinline__ void split3(float v, uint32_t &hi, uint32_t &mid, uint32_t &lo) {
  hi = __float_as_uint(v) & 0xFFFF0000u;
  const float r = v - __uint_as_float(hi);                         // exact
  mid = __float_as_uint(r) & 0xFFFF0000u;
  lo = __float_as_uint(r - __uint_as_float(mid)) & 0xFFFF0000u;    // exact, <= 8 bits
}

template <bool TN>
__device__ __forceinline__ void stage_skinny(uint16_t *xs, int sc, int kq,
                                             const float4 (&x)[B16Lds<TN>::XL]) {
  using Lds = B16Lds<TN>;
  uint16_t *base = xs + sc * Lds::CS + 4 * Lds::XL * kq;
#pragma unroll
  for (int g = 0; g < Lds::XL; ++g) {
    const float v[4] = {x[g].x, x[g].y, x[g].z, x[g].w};
    uint32_t hi[4], mid[4], lo[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) split3(v[i], hi[i], mid[i], lo[i]);
    *reinterpret_cast<uint2 *>(base + 4 * g) = make_uint2((hi[0] >> 16) | hi[1], (hi[2] >> 16) | hi[3]);
    *reinterpret_cast<uint2 *>(base + 4 * g + Lds::PLANE) =
        make_uint2((mid[0] >> 16) | mid[1], (mid[2] >> 16) | mid[3]);
    *reinterpret_cast<uint2 *>(base + 4 * g + 2 * Lds::PLANE) =
        make_uint2((lo[0] >> 16) | lo[1], (lo[2] >> 16) | lo[3]);
  }
}

template <bool TN>
__device__ __forceinline__ void mma_slice_bf16(floatx4 (&acc)[16], const ASlot<TN> &s,
                                               const uint16_t *xs, int li, int lk) {
  using Lds = B16Lds<TN>;
  constexpr int KS = B16Cfg<TN>::SL / 32;
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

template <bool TN, bool AVEC>
__global__ __launch_bounds__(kB16Threads) void gemm_bf16_kernel(
    const uint16_t *A, int64_t lda, const float *xt, int64_t kp, float *__restrict__ C, int64_t ldc,
    int64_t M, int64_t N, int64_t K, int64_t kps, int64_t tiles, int64_t total, float alpha,
    float beta, float *__restrict__ part, int64_t mclamp) {
  using Cfg = B16Cfg<TN>;
  using Lds = B16Lds<TN>;
  constexpr int SL = Cfg::SL, RING = Cfg::RING, NBUF = Cfg::NBUF, XL = Lds::XL;
  __shared__ __attribute__((aligned(16))) uint16_t xs[NBUF][Lds::STAGE];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t L = b16_xcd_remap(blockIdx.x, total);
  const int64_t tile = L % tiles, split = L / tiles;
  const int64_t t0 = tile * kB16Rows + 64 * wave;
  const int64_t kb = split * kps;
  const int64_t ke = (kb + kps < K) ? kb + kps : K;
  // slices of this split, a multiple of RING (kps is a multiple of kKGroup;
  // slices past K meet zero skinny rows)
  const int64_t nsl = ((ke - kb + kKGroup - 1) / kKGroup) * RING;
  const int sc = tid >> 3, kq = tid & 7;
  const float *xsrc = xt + sc * kp + kb + 4 * XL * kq;

  floatx4 acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};

  ASlot<TN> ar[RING];
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
    load_slot<TN, AVEC>(A, lda, M, K, t0, li, lk, kb + sl * SL, ar[slot], mclamp);
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  };
#pragma unroll
  for (int d = 0; d < RING; ++d) issue(d, d);
  stage_skinny<TN>(xs[0], sc, kq, xr[0]);

  for (int64_t s0 = 0; s0 < nsl; s0 += RING) {
#pragma unroll
    for (int d = 0; d < RING; ++d) {
      // RING is a multiple of NBUF: slice s0 + d lives in buffer d % NBUF
      const int buf = d % NBUF;
      __syncthreads();                 // slice s0 + d staged; slice s0 + d - 1 consumed
      __builtin_amdgcn_sched_barrier(0);
      mma_slice_bf16<TN>(acc, ar[d], xs[buf], li, lk);
      __builtin_amdgcn_sched_barrier(0);
      stage_skinny<TN>(xs[(d + 1) % NBUF], sc, kq, xr[(d + 1) % RING]);
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

// ------------------------------------------------------------------ host
static int64_t bf16_slots(int is_tn) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, int64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair(dev, is_tn);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  const void *fn = is_tn ? reinterpret_cast<const void *>(&gemm_bf16_kernel<true, true>)
                         : reinterpret_cast<const void *>(&gemm_bf16_kernel<false, true>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kB16Threads, 0) != hipSuccess ||
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
int gemm_bf16_choose_ksplit(int64_t M, int64_t K, int is_tn, int64_t max_split) {
  if (M < 1 || K < 1) return 1;
  const int64_t tiles = (M + kB16Rows - 1) / kB16Rows;
  const int64_t slots = bf16_slots(is_tn);
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

size_t bf16_pack_bytes(int64_t K) { return (size_t)bf16_padded_k(K) * kBld * sizeof(float); }

template <bool TN>
static int launch_bf16(const uint16_t *A, int64_t lda, const float *X, int64_t ldx, float *C,
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
  const int64_t tiles = (M + kB16Rows - 1) / kB16Rows;
  const int64_t total = tiles * nsp;
  const uintptr_t ad = reinterpret_cast<uintptr_t>(A);
  // vector loads: 8-byte (TN) / 16-byte (NN) aligned rows whose groups of 4
  // columns (TN) / 8 k (NN) stay inside the row or its padding up to lda
  const int64_t m4 = (M + 3) / 4 * 4, k8 = (K + 7) / 8 * 8;
  const bool avec = TN ? (M >= 4 && lda % 4 == 0 && (ad & 7) == 0 && (M % 4 == 0 || lda >= m4))
                       : (K >= 8 && lda % 8 == 0 && (ad & 15) == 0 && (K % 8 == 0 || lda >= k8));
  const int64_t mclamp = (TN && M % 4 != 0) ? m4 : M;
  dim3 grid((unsigned)total), blk(kB16Threads);
  if (avec)
    hipLaunchKernelGGL((gemm_bf16_kernel<TN, true>), grid, blk, 0, st, A, lda, xt, kp, C, ldc, M, N,
                       K, kps, tiles, total, alpha, beta, p, mclamp);
  else
    hipLaunchKernelGGL((gemm_bf16_kernel<TN, false>), grid, blk, 0, st, A, lda, xt, kp, C, ldc, M,
                       N, K, kps, tiles, total, alpha, beta, p, mclamp);
  return nsp;
}

int launch_gemm_bf16_nn_main(const uint16_t *A, int64_t lda, const float *X, int64_t ldx, float *C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                             int ksplit, float *part, float *xt, hipStream_t st) {
  return launch_bf16<false>(A, lda, X, ldx, C, ldc, M, N, K, alpha, beta, ksplit, part, xt, st);
}

int launch_gemm_bf16_tn_main(const uint16_t *A, int64_t lda, const float *Y, int64_t ldy, float *C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha, float beta,
                             int ksplit, float *part, float *xt, hipStream_t st) {
  return launch_bf16<true>(A, lda, Y, ldy, C, ldc, M, N, K, alpha, beta, ksplit, part, xt, st);
}

}  // namespace farpca_int
