// Test-matrix generation on the fly (Definitions 2.1-2.4; the fixed-count
// sparse sign variant named after Definition 2.2).  One workgroup per chunk of
// 64 rows of Omega_j (= 64 columns of A); one thread per row.
//
// Outputs per row r:   mask word (nonzero columns), negative-sign word
//                      (bit c set iff entry (r, c) < 0), dense row (FP32;
//                      only if dense_out is given).
// Outputs per chunk:   column lists (ascending row inside each column) that
//                      the sketch kernel walks: colptr[c] .. colptr[c+1].
#include "internal.h"
#include "philox_dev.h"

namespace farpca_int {
using namespace farpca_dev;

__global__ __launch_bounds__(64) void omega_kernel(OmegaSpec s, int64_t n, int64_t block_j,
                                                   uint64_t *__restrict__ mask_out,
                                                   uint64_t *__restrict__ sign_out,
                                                   float *__restrict__ dense_out,
                                                   uint32_t *__restrict__ colptr,
                                                   ChunkEntry *__restrict__ entries,
                                                   int lds_stride) {
  __shared__ float rval[kChunk][kMaxBlock + 1];

  const int t = threadIdx.x;
  const int64_t chunk = blockIdx.x;
  const int64_t r = chunk * kChunk + t;
  const int b = s.b;
  uint64_t mask = 0, neg = 0;

  if (r < n) {
    const uint64_t row = (uint64_t)r, blk = (uint64_t)block_j;
    if (s.kind == SK_SPARSE_SIGN && s.zeta > 0) {
      // Floyd's sampling of zeta distinct columns out of b.
      uint64_t chosen = 0;
      // 32-bit draw q is half of word (q / 2) % 4 of call q / 8: one call
      // serves 8 draws
      u64x4 w8 = philox4x64_10(row, blk, 0, 0, s.seed, 0);
      for (int q = 0; q < s.zeta; ++q) {
        const uint32_t jj = (uint32_t)(b - s.zeta + q);
        if (q > 0 && (q & 7) == 0) w8 = philox4x64_10(row, blk, 0, (uint64_t)(q >> 3), s.seed, 0);
        const uint64_t word = pick64(w8, (uint32_t)(q >> 1) & 3u);
        const uint32_t u = (q & 1) ? (uint32_t)(word >> 32) : (uint32_t)(word & 0xFFFFFFFFull);
        const uint32_t tt = (uint32_t)(((uint64_t)u * (uint64_t)(jj + 1u)) >> 32);
        if ((chosen >> tt) & 1ull) chosen |= 1ull << jj; else chosen |= 1ull << tt;
      }
      const uint64_t w = draw64(s.seed, row, blk, 1, 0);
      int k = 0;
      for (int c = 0; c < b; ++c) {
        if ((chosen >> c) & 1ull) {
          if ((w >> k) & 1ull) neg |= 1ull << c;
          ++k;
        }
      }
      mask = chosen;
    } else if (s.kind == SK_GAUSSIAN) {
      mask = (b == 64) ? ~0ull : ((1ull << b) - 1ull);
    } else {
      // i.i.d. mask: entry (r, c) nonzero iff 32-bit draw c < T(p).
      for (int c0 = 0; c0 < b; c0 += 8) {
        const u64x4 w = philox4x64_10(row, blk, 0, (uint64_t)(c0 >> 3), s.seed, 0);
#pragma unroll
        for (int h = 0; h < 8; ++h) {
          const int c = c0 + h;
          const uint64_t word = w.v[h >> 1];
          const uint32_t u = (h & 1) ? (uint32_t)(word >> 32) : (uint32_t)(word & 0xFFFFFFFFull);
          if (c < b && u < s.thr) mask |= 1ull << c;
        }
      }
      if (s.kind == SK_SPARSE_SIGN) neg = draw64(s.seed, row, blk, 1, 0) & mask;
    }
    // Unscaled values (what the sketch accumulates) and the dense copy
    // (values computed in FP64, rounded once).
    float *drow = dense_out ? dense_out + r * (int64_t)kBld : nullptr;
    uint64_t negative = 0;
    for (int c = 0; c < b; ++c) {
      double v = 0.0, dv = 0.0;
      const bool on = (mask >> c) & 1ull;
      switch (s.kind) {
        case SK_GAUSSIAN: v = gaussian_entry(s.seed, row, blk, (uint32_t)c); dv = v; break;
        case SK_SPARSE_GAUSSIAN:
          if (on) { v = gaussian_entry(s.seed, row, blk, (uint32_t)c); dv = v * s.dense_scale; }
          break;
        case SK_SPARSE_SIGN:
          if (on) { v = ((neg >> c) & 1ull) ? -1.0 : 1.0; dv = v * s.dense_scale; }
          break;
        case SK_STD_BERNOULLI: v = on ? 1.0 : 0.0; dv = v - s.p; break;
        default: v = on ? 1.0 : 0.0; dv = v; break;
      }
      rval[t][c] = (float)v;
      if (drow) drow[c] = (float)dv;
      if (dv < 0.0) negative |= 1ull << c;
    }
    if (drow)
      for (int c = b; c < kBld; ++c) drow[c] = 0.0f;
    mask_out[r] = mask;
    sign_out[r] = negative;
  }
  __syncthreads();                   // rval complete
  if (colptr == nullptr) return;

  // Column lists of this chunk: thread t owns column c = t.  The rows of
  // column c are the lanes whose mask has bit c: one ballot per column gives
  // them as a bit set (ascending rows = ascending bits); the starts are an
  // exclusive prefix sum over the lanes.
  const int c = t;
  uint64_t colbits = 0;
  for (int cc = 0; cc < kMaxBlock; ++cc) {
    const uint64_t bal = __ballot(((mask >> cc) & 1ull) != 0ull);
    if (c == cc) colbits = bal;
  }
  uint32_t cnt = 0;
  if (c < b) {
    cnt = (uint32_t)__popcll(colbits);
    cnt = (cnt + kListPad - 1) / kListPad * kListPad;     // padded to whole groups
  }
  uint32_t incl = cnt;
#pragma unroll
  for (int off = 1; off < kMaxBlock; off <<= 1) {
    const uint32_t v = __shfl_up(incl, off, kMaxBlock);
    if (t >= off) incl += v;
  }
  const uint32_t start = incl - cnt;
  uint32_t *cp = colptr + chunk * (kMaxBlock + 1);
  cp[c] = start;
  if (t == kMaxBlock - 1) cp[kMaxBlock] = incl;
  if (c < b) {
    ChunkEntry *ent = entries + chunk * (int64_t)kEntCap;
    uint32_t pos = start;
    uint64_t rows = colbits;
    while (rows) {
      const int k = __ffsll((long long)rows) - 1;
      rows &= rows - 1ull;
      ChunkEntry e;
      e.lds_off = (uint32_t)(k * lds_stride);
      e.val = rval[k][c];
      ent[pos++] = e;
    }
    const ChunkEntry pad = {0u, 0.0f};      // adds 0 * A[i, first column]: exact no-op
    while (pos < start + cnt) ent[pos++] = pad;
  }
}

void launch_omega(const OmegaSpec &s, int64_t n, int64_t block_j, uint64_t *mask_out,
                  uint64_t *sign_out, float *dense_out, uint32_t *colptr, ChunkEntry *entries,
                  int lds_row_stride_bytes, hipStream_t st) {
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(omega_kernel, dim3((unsigned)nchunks), dim3(kChunk), 0, st, s, n, block_j,
                     mask_out, sign_out, dense_out, colptr, entries, lds_row_stride_bytes);
}

}  // namespace farpca_int
