// Sparse sketch S = A * Omega_j for the sparse test matrices (Section 3: the
// cost of A B_j is nnz(B_j) m instead of a dense product).
//
// Four waves per workgroup; lane i of wave w owns row i0 + 64 w + i of A.  For
// each chunk of 64 columns of A the workgroup stages the chunk's column lists
// in LDS (shared by the four waves) and each wave
//   1. reads the 64 x 64 tile with coalesced 16-byte loads (4 rows per
//      instruction, 256 contiguous bytes per row) and stores it transposed into
//      LDS (stride 65 floats: conflict-free stores and loads),
//   2. walks the chunk's column lists (ascending row inside each output
//      column, padded with zero entries to groups of four; every lane reads
//      the same entry, an LDS broadcast), a group at a time so the LDS reads
//      overlap, and accumulates
//      acc[c] += val * tile[r][lane] - each A element is read from HBM once
//      and from LDS once per nonzero of its Omega row.
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

constexpr int kSketchWaves = 4;      // waves per workgroup (each owns 64 rows of A)
constexpr int kPiece = 1024;         // column-list entries staged in LDS at a time

template <bool VEC, bool DIRECT>
__global__ __launch_bounds__(64 * kSketchWaves, 2) void sketch_kernel(
    const float *__restrict__ A, int64_t lda, int64_t m, int64_t n, int b,
    const uint32_t *__restrict__ colptr, const ChunkEntry *__restrict__ entries,
    float *__restrict__ out, int64_t chunks_per_split, float scale, const float *__restrict__ z,
    float zc) {
  __shared__ float tiles[kSketchWaves][kChunk * kTileStride];
  __shared__ uint2 ents[kPiece];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * (64 * kSketchWaves) + 64 * wave;
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  const int64_t ch_begin = (int64_t)blockIdx.y * chunks_per_split;
  int64_t ch_end = ch_begin + chunks_per_split;
  if (ch_end > nchunks) ch_end = nchunks;
  float *tile = tiles[wave];
  const char *tile_bytes = reinterpret_cast<const char *>(tile) + lane * 4;

  float acc[kMaxBlock];
#pragma unroll
  for (int c = 0; c < kMaxBlock; ++c) acc[c] = 0.0f;

  // A tile and column bounds of the next chunk are loaded one chunk ahead
  float4 reg[16];
  uint32_t cp_next = 0;
  if (ch_begin < ch_end) {
    load_tile_regs<VEC>(A, lda, m, n, i0, ch_begin * kChunk, lane, reg);
    cp_next = colptr[ch_begin * (kMaxBlock + 1) + lane];
  }

  for (int64_t ch = ch_begin; ch < ch_end; ++ch) {
    __syncthreads();
    store_tile_lds(tile, lane, reg);
    const uint32_t cp_lane = cp_next;                      // lane c holds the start of column c
    const uint32_t total = colptr[ch * (kMaxBlock + 1) + kMaxBlock];
    if (ch + 1 < ch_end) {
      load_tile_regs<VEC>(A, lda, m, n, i0, (ch + 1) * kChunk, lane, reg);
      cp_next = colptr[(ch + 1) * (kMaxBlock + 1) + lane];
    }
    const uint2 *ent_g = reinterpret_cast<const uint2 *>(entries + ch * (int64_t)kEntCap);
    for (uint32_t p0 = 0; p0 < total; p0 += kPiece) {
      const uint32_t p1 = (total - p0 > (uint32_t)kPiece) ? p0 + kPiece : total;
      if (p0 > 0) __syncthreads();
      for (uint32_t e = p0 + tid; e < p1; e += 64 * kSketchWaves) ents[e - p0] = ent_g[e];
      __syncthreads();
#pragma unroll
      for (int c = 0; c < kMaxBlock; ++c) {
        if (c < b) {
          // this column's entries inside the staged piece [p0, p1); list
          // starts, ends and piece bounds are multiples of kListPad
          const uint32_t c0 = __builtin_amdgcn_readlane(cp_lane, c);
          const uint32_t c1 = (c + 1 < kMaxBlock) ? __builtin_amdgcn_readlane(cp_lane, c + 1) : total;
          const uint32_t lo = c0 > p0 ? c0 : p0;
          const uint32_t hi = c1 < p1 ? c1 : p1;
          if (lo < hi) {
            float a = acc[c];
            for (uint32_t e = lo - p0; e < hi - p0; e += kListPad) {   // 0 <= e < e + 4 <= kPiece
              uint2 q[kListPad];
              float x[kListPad];
#pragma unroll
              for (int u = 0; u < kListPad; ++u) q[u] = ents[e + u];
#pragma unroll
              for (int u = 0; u < kListPad; ++u) x[u] = *reinterpret_cast<const float *>(tile_bytes + q[u].x);
#pragma unroll
              for (int u = 0; u < kListPad; ++u) a = fmaf(__uint_as_float(q[u].y), x[u], a);
            }
            acc[c] = a;
          }
        }
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
  const int rows_wg = 64 * kSketchWaves;
  dim3 grid((unsigned)((m + rows_wg - 1) / rows_wg), (unsigned)nsplit);
  dim3 blk(64 * kSketchWaves);
  if (nsplit == 1) {
    if (vec) hipLaunchKernelGGL((sketch_kernel<true, true>), grid, blk, 0, st, A, lda, m, n, b,
                                colptr, entries, out, cps, scale, z, zc);
    else hipLaunchKernelGGL((sketch_kernel<false, true>), grid, blk, 0, st, A, lda, m, n, b,
                            colptr, entries, out, cps, scale, z, zc);
  } else {
    if (vec) hipLaunchKernelGGL((sketch_kernel<true, false>), grid, blk, 0, st, A, lda, m, n, b,
                                colptr, entries, out, cps, scale, z, zc);
    else hipLaunchKernelGGL((sketch_kernel<false, false>), grid, blk, 0, st, A, lda, m, n, b,
                            colptr, entries, out, cps, scale, z, zc);
  }
}

int sketch_choose_split(int64_t m, int64_t n) {
  const int64_t tiles = (m + 64 * kSketchWaves - 1) / (64 * kSketchWaves);
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  int64_t s = (512 + tiles - 1) / tiles;    // about 512 workgroups (2 per CU)
  if (s < 1) s = 1;
  if (s > nchunks) s = nchunks;
  if (s > 16) s = 16;
  return (int)s;
}

}  // namespace farpca_int
