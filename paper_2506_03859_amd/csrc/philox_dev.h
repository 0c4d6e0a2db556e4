// Device-side Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the draw
// layout of the random test matrices (Definitions 2.1-2.4 of the paper).
//
// Counter (row r, block j, purpose, t), key (seed, 0); a call yields four
// 64-bit words.  64-bit draw q of (r, j, purpose) is word q % 4 of call
// t = q / 4; 32-bit draw q is the low (even q) / high (odd q) half of 64-bit
// draw q / 2.  Purposes: 0 mask/index draws, 1 sign word, 2 Box-Muller pairs.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace farpca_dev {

struct u64x4 { uint64_t v[4]; };

__device__ __forceinline__ void mul_hilo64(uint64_t a, uint64_t b, uint64_t &hi, uint64_t &lo) {
  lo = a * b;
  hi = __umul64hi(a, b);
}

__device__ __forceinline__ u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t hi0, lo0, hi1, lo1;
    mul_hilo64(M0, c0, hi0, lo0);
    mul_hilo64(M1, c2, hi1, lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  u64x4 out; out.v[0] = c0; out.v[1] = c1; out.v[2] = c2; out.v[3] = c3;
  return out;
}

// 64-bit draw q for (row, block, purpose).
__device__ __forceinline__ uint64_t draw64(uint64_t seed, uint64_t row, uint64_t block,
                                           uint64_t purpose, uint32_t q) {
  u64x4 w = philox4x64_10(row, block, purpose, q >> 2, seed, 0);
  const uint32_t s = q & 3u;
  return s == 0 ? w.v[0] : (s == 1 ? w.v[1] : (s == 2 ? w.v[2] : w.v[3]));
}

__device__ __forceinline__ uint32_t draw32(uint64_t seed, uint64_t row, uint64_t block,
                                           uint64_t purpose, uint32_t q) {
  uint64_t w = draw64(seed, row, block, purpose, q >> 1);
  return (q & 1u) ? (uint32_t)(w >> 32) : (uint32_t)(w & 0xFFFFFFFFull);
}

__device__ __forceinline__ uint64_t pick64(const u64x4 &w, uint32_t s) {
  return s == 0 ? w.v[0] : (s == 1 ? w.v[1] : (s == 2 ? w.v[2] : w.v[3]));
}

// Box-Muller standard normal for entry (row, col) of block `block`, in FP64.
// Its two 64-bit draws 2 col and 2 col + 1 are words 2 (col % 2) and
// 2 (col % 2) + 1 of one call (t = col / 2).
__device__ __forceinline__ double gaussian_entry(uint64_t seed, uint64_t row, uint64_t block, uint32_t col) {
  const u64x4 w = philox4x64_10(row, block, 2, col >> 1, seed, 0);
  const uint64_t w1 = (col & 1u) ? w.v[2] : w.v[0];
  const uint64_t w2 = (col & 1u) ? w.v[3] : w.v[1];
  const double u1 = ((double)(w1 >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(w2 >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

}  // namespace farpca_dev
