// Sparse sketch S = A * Omega_j for the sparse test matrices (Section 3: the
// cost of A B_j is nnz(B_j) m instead of a dense product).
//
// One wave per workgroup; lane i owns row i0 + i of A.  For each chunk of 64
// columns of A the wave
//   1. reads the 64 x 64 tile with coalesced 16-byte loads (4 rows per
//      instruction, 256 contiguous bytes per row) and stores it transposed into
//      LDS (stride 65 floats: conflict-free stores and loads),
//   2. walks the chunk's column lists (ascending row inside each output
//      column; the lists are wave-uniform, read through the scalar cache) and
//      accumulates acc[c] += val * tile[r][lane] - each A element is read from
//      HBM once and from LDS once per nonzero of its Omega row.
// The next chunk's tile is loaded into registers while the current one is
// processed.  Sums run in a fixed order, so results are bitwise repeatable;
// the +-1 values of the sign sketches are added exactly (no scaling until the
// final multiply).  Chunks are split into `nsplit` consecutive groups (grid y)
// to fill the GPU when m is small; the partial sums are then reduced in a
// fixed order by reduce_partials.
#include "internal.h"

namespace farpca_int {

constexpr int kTileStride = kChunk + 1;   // floats per LDS row of the staged tile

int sketch_lds_row_stride_bytes() { return kTileStride * 4; }
int sketch_rows_per_wg() { return 64; }

template <bool VEC>
__device__ __forceinline__ void load_tile_regs(const float *__restrict__ A, int64_t lda,
                                               int64_t m, int64_t n, int64_t i0, int64_t col0,
                                               int lane, float4 (&reg)[16]) {
  // instruction q covers rows i0 + 4q + lane/16, columns col0 + 4*(lane%16) .. +3
  const int rsub = lane >> 4;
  const int c4 = (lane & 15) * 4;
  const int64_t col = col0 + c4;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t row = i0 + 4 * q + rsub;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (row < m) {
      const float *p = A + row * lda + col;
      if (VEC && col + 3 < n) {
        v = *reinterpret_cast<const float4 *>(p);
      } else {
        if (col + 0 < n) v.x = p[0];
        if (col + 1 < n) v.y = p[1];
        if (col + 2 < n) v.z = p[2];
        if (col + 3 < n) v.w = p[3];
      }
    }
    reg[q] = v;
  }
}

__device__ __forceinline__ void store_tile_lds(float *tile, int lane, const float4 (&reg)[16]) {
  const int rsub = lane >> 4;
  const int c4 = (lane & 15) * 4;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int row = 4 * q + rsub;
    tile[(c4 + 0) * kTileStride + row] = reg[q].x;
    tile[(c4 + 1) * kTileStride + row] = reg[q].y;
    tile[(c4 + 2) * kTileStride + row] = reg[q].z;
    tile[(c4 + 3) * kTileStride + row] = reg[q].w;
  }
}

template <bool VEC, bool DIRECT>
__global__ __launch_bounds__(64) void sketch_kernel(const float *__restrict__ A, int64_t lda,
                                                    int64_t m, int64_t n, int b,
                                                    const uint32_t *__restrict__ colptr,
                                                    const ChunkEntry *__restrict__ entries,
                                                    float *__restrict__ out, int64_t chunks_per_split,
                                                    float scale, const float *__restrict__ z,
                                                    float zc) {
  __shared__ float tile[kChunk * kTileStride];
  const int lane = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  const int64_t ch_begin = (int64_t)blockIdx.y * chunks_per_split;
  int64_t ch_end = ch_begin + chunks_per_split;
  if (ch_end > nchunks) ch_end = nchunks;

  float acc[kMaxBlock];
#pragma unroll
  for (int c = 0; c < kMaxBlock; ++c) acc[c] = 0.0f;

  float4 reg[16];
  if (ch_begin < ch_end) load_tile_regs<VEC>(A, lda, m, n, i0, ch_begin * kChunk, lane, reg);
  const char *tile_bytes = reinterpret_cast<const char *>(tile) + lane * 4;

  for (int64_t ch = ch_begin; ch < ch_end; ++ch) {
    __syncthreads();
    store_tile_lds(tile, lane, reg);
    __syncthreads();
    if (ch + 1 < ch_end) load_tile_regs<VEC>(A, lda, m, n, i0, (ch + 1) * kChunk, lane, reg);

    const uint32_t *cp = colptr + ch * (kMaxBlock + 1);
    const ChunkEntry *ent = entries + ch * (int64_t)(kChunk * kMaxBlock);
#pragma unroll
    for (int c = 0; c < kMaxBlock; ++c) {
      if (c < b) {
        const uint32_t e0 = cp[c], e1 = cp[c + 1];
        float a = acc[c];
        uint32_t e = e0;
        for (; e + 4 <= e1; e += 4) {
          const ChunkEntry q0 = ent[e], q1 = ent[e + 1], q2 = ent[e + 2], q3 = ent[e + 3];
          const float x0 = *reinterpret_cast<const float *>(tile_bytes + q0.lds_off);
          const float x1 = *reinterpret_cast<const float *>(tile_bytes + q1.lds_off);
          const float x2 = *reinterpret_cast<const float *>(tile_bytes + q2.lds_off);
          const float x3 = *reinterpret_cast<const float *>(tile_bytes + q3.lds_off);
          a = fmaf(q0.val, x0, a);
          a = fmaf(q1.val, x1, a);
          a = fmaf(q2.val, x2, a);
          a = fmaf(q3.val, x3, a);
        }
        for (; e < e1; ++e) {
          const ChunkEntry q0 = ent[e];
          a = fmaf(q0.val, *reinterpret_cast<const float *>(tile_bytes + q0.lds_off), a);
        }
        acc[c] = a;
      }
    }
  }

  const int64_t row = i0 + lane;
  if (row >= m) return;
  if (DIRECT) {
    float *o = out + row * (int64_t)kBld;
    const float zr = z ? zc * z[row] : 0.0f;
#pragma unroll
    for (int c = 0; c < kMaxBlock; ++c) o[c] = (c < b) ? fmaf(scale, acc[c], zr) : 0.0f;
  } else {
    float *o = out + ((int64_t)blockIdx.y * m + row) * (int64_t)kBld;
#pragma unroll
    for (int c = 0; c < kMaxBlock; ++c) o[c] = (c < b) ? acc[c] : 0.0f;
  }
}

// part: nsplit == 1 -> final S (scale, z applied); else partials (nsplit x m x kBld).
void launch_sketch_full(const float *A, int64_t lda, int64_t m, int64_t n, int b,
                        const uint32_t *colptr, const ChunkEntry *entries, float *out,
                        int nsplit, float scale, const float *z, float zc, hipStream_t st) {
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  if (nsplit < 1) nsplit = 1;
  if (nsplit > nchunks) nsplit = (int)nchunks;
  const int64_t cps = (nchunks + nsplit - 1) / nsplit;
  nsplit = (int)((nchunks + cps - 1) / cps);
  const bool vec = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  dim3 grid((unsigned)((m + 63) / 64), (unsigned)nsplit);
  if (nsplit == 1) {
    if (vec) hipLaunchKernelGGL((sketch_kernel<true, true>), grid, dim3(64), 0, st, A, lda, m, n, b,
                                colptr, entries, out, cps, scale, z, zc);
    else hipLaunchKernelGGL((sketch_kernel<false, true>), grid, dim3(64), 0, st, A, lda, m, n, b,
                            colptr, entries, out, cps, scale, z, zc);
  } else {
    if (vec) hipLaunchKernelGGL((sketch_kernel<true, false>), grid, dim3(64), 0, st, A, lda, m, n, b,
                                colptr, entries, out, cps, scale, z, zc);
    else hipLaunchKernelGGL((sketch_kernel<false, false>), grid, dim3(64), 0, st, A, lda, m, n, b,
                            colptr, entries, out, cps, scale, z, zc);
  }
}

int sketch_choose_split(int64_t m, int64_t n) {
  const int64_t tiles = (m + 63) / 64;
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  int64_t s = (2048 + tiles - 1) / tiles;   // about 2048 waves in flight
  if (s < 1) s = 1;
  if (s > nchunks) s = nchunks;
  if (s > 16) s = 16;
  return (int)s;
}

}  // namespace farpca_int
