// Sparse sketch S = A * Omega_j for the sparse test matrices (Section 3: the
// cost of A B_j is nnz(B_j) m instead of a dense product).
//
// Four waves per workgroup; lane i of wave w owns row i0 + 64 w + i of A.  A
// is streamed in chunks of 64 columns.  Per chunk each wave
//   1. holds the chunk's 64 x 64 tile of A in registers (16-byte loads, 4
//      rows x 256 contiguous bytes per instruction), fetched while the
//      previous chunk is being processed, and stores it transposed into its
//      own LDS tile (stride 65 floats: conflict-free stores and loads);
//   2. walks the chunk's column lists of Omega (staged in LDS once for the
//      four waves, padded per column to groups of four, every lane reading
//      the same entry: an LDS broadcast) four output columns at a time, so
//      that 16 independent tile reads are in flight per step, with the next
//      step's entries already being read, accumulating
//      acc[c] += val * tile[r][lane]: each A element is read from HBM once
//      and from LDS once per nonzero of its Omega row.
// A column whose list is exhausted inside a step reads a group of zero
// entries (0 * finite = +0, an exact no-op).  Each column's sum runs in list
// order, so results are bitwise repeatable; the +-1 values of the sign
// sketches are added exactly (no scaling until the final multiply).  Chunks
// are split into consecutive groups (K splits) to fill the GPU; the partial
// sums are reduced in split order by reduce_partials.
#include <map>
#include <mutex>

#include "internal.h"

namespace farpca_int {

constexpr int kTileStride = kChunk + 1;   // floats per LDS row of the staged tile
constexpr int kSketchWaves = 4;           // waves per workgroup (each owns 64 rows of A)
constexpr int kPiece = 768;               // column-list entries staged in LDS at a time
constexpr int kPieceLoads = kPiece / (64 * kSketchWaves);   // entries per thread per piece
static_assert(kPiece % (64 * kSketchWaves) == 0, "piece must split evenly over the threads");
static_assert(kPiece % kListPad == 0, "pieces hold whole groups");

int sketch_lds_row_stride_bytes() { return kTileStride * 4; }
int sketch_rows_per_wg() { return 64 * kSketchWaves; }

// Chunk tile of A into registers: instruction q covers rows i0 + 4q + lane/16,
// columns col0 + 4 (lane%16) .. +3.  FAST: all 64 rows inside m, the chunk
// inside n, rows 16-byte aligned.  Otherwise addresses are clamped into A and
// columns beyond n zeroed (rows beyond m feed outputs that are never stored).
template <bool FAST>
__device__ __forceinline__ void load_tile(const float *__restrict__ A, int64_t lda, int64_t m,
                                          int64_t n, int64_t i0, int64_t col0, int lane,
                                          float4 (&reg)[16]) {
  const int rsub = lane >> 4;
  const int64_t col = col0 + (lane & 15) * 4;
  // FAST: a uniform row base per instruction plus a 32-bit lane offset
  // (lda < 2^28), so the address arithmetic stays scalar
  const int32_t loff = rsub * (int32_t)lda + (lane & 15) * 4;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int64_t row = i0 + 4 * q + rsub;
    if (FAST) {
      const float *rb = A + (i0 + 4 * q) * lda + col0;
      reg[q] = *reinterpret_cast<const float4 *>(rb + loff);
    } else {
      const float *p = A + (row < m ? row : m - 1) * lda;
      float v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float u = p[col + t < n ? col + t : n - 1];
        v[t] = (col + t < n) ? u : 0.0f;
      }
      reg[q] = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
}

__device__ __forceinline__ void store_tile(float *tile, int lane, const float4 (&reg)[16]) {
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

// Logical workgroup id (see gemm.hip): XCD x runs physical ids 8 j + x; the
// regrouping gives it a contiguous range of logical ids, i.e. one K split.
__device__ __forceinline__ int64_t sketch_xcd_remap(int64_t g, int64_t T) {
  const int64_t T8 = T & ~int64_t(7);
  if (g >= T8) return g;
  return (g & 7) * (T8 >> 3) + (g >> 3);
}

// Entries [p0, p1) of one chunk staged in E (relative index), E[kPiece ..
// kPiece + 3] zero.  Adds them into acc four columns at a time; the entries
// of step k + 1 are read before the tile reads of step k.
__device__ __forceinline__ void sketch_piece(float (&acc)[kMaxBlock], const uint2 *E,
                                             const char *tile_bytes, uint32_t cp_lane,
                                             uint32_t total, uint32_t p0, uint32_t p1, int b) {
#pragma unroll
  for (int cq = 0; cq < kMaxBlock; cq += 4) {
    if (cq < b) {
      uint32_t lo[4], len[4];
      uint32_t kmax = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = cq + i;
        const uint32_t c0 = __builtin_amdgcn_readlane(cp_lane, c);
        const uint32_t c1 = (c + 1 < kMaxBlock) ? __builtin_amdgcn_readlane(cp_lane, c + 1) : total;
        const uint32_t l0 = c0 > p0 ? c0 : p0;
        const uint32_t h0 = c1 < p1 ? c1 : p1;
        len[i] = h0 > l0 ? h0 - l0 : 0u;      // a multiple of kListPad
        lo[i] = h0 > l0 ? l0 - p0 : 0u;
        kmax = len[i] > kmax ? len[i] : kmax;
      }
      if (kmax == 0) continue;
      float a[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = acc[cq + i];
      // entries of step k (past a column's end: the zero group)
      auto read_entries = [&](uint32_t k, uint2 (&q)[4][kListPad]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t base = (k < len[i]) ? lo[i] + k : (uint32_t)kPiece;   // + 3 < kPiece + 4
#pragma unroll
          for (int u = 0; u < kListPad; ++u) q[i][u] = E[base + u];
        }
      };
      auto accumulate = [&](const uint2 (&q)[4][kListPad]) {
        float x[4][kListPad];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < kListPad; ++u) x[i][u] = *reinterpret_cast<const float *>(tile_bytes + q[i][u].x);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int u = 0; u < kListPad; ++u) a[i] = fmaf(__uint_as_float(q[i][u].y), x[i][u], a[i]);
      };
      uint2 qa[4][kListPad], qb[4][kListPad];
      read_entries(0, qa);
      for (uint32_t k = 0; k < kmax; k += 2 * kListPad) {
        read_entries(k + kListPad, qb);         // zero group once past kmax
        accumulate(qa);
        if (k + kListPad >= kmax) break;
        read_entries(k + 2 * kListPad, qa);
        accumulate(qb);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[cq + i] = a[i];
    }
  }
}

template <bool VEC, bool DIRECT>
__global__ __launch_bounds__(64 * kSketchWaves, 2) void sketch_kernel(
    const float *__restrict__ A, int64_t lda, int64_t m, int64_t n, int b,
    const uint32_t *__restrict__ colptr, const ChunkEntry *__restrict__ entries,
    float *__restrict__ out, int64_t chunks_per_split, int64_t tiles, int64_t total_wg,
    float scale, const float *__restrict__ z, float zc) {
  __shared__ float tiles_lds[kSketchWaves][kChunk * kTileStride];
  __shared__ uint2 ents[2][kPiece + kListPad];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t L = sketch_xcd_remap(blockIdx.x, total_wg);
  const int64_t tile = L % tiles, split = L / tiles;
  const int64_t i0 = tile * (64 * kSketchWaves) + 64 * wave;
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  const int64_t ch_begin = split * chunks_per_split;
  int64_t ch_end = ch_begin + chunks_per_split;
  if (ch_end > nchunks) ch_end = nchunks;
  float *tile_lds = tiles_lds[wave];
  const char *tile_bytes = reinterpret_cast<const char *>(tile_lds) + lane * 4;
  const bool rows_in = VEC && (i0 + 64 <= m);

  if (tid < 2 * kListPad) ents[tid / kListPad][kPiece + tid % kListPad] = make_uint2(0u, 0u);

  float acc[kMaxBlock];
#pragma unroll
  for (int c = 0; c < kMaxBlock; ++c) acc[c] = 0.0f;

  // next chunk in registers: A tile, first piece of its entries, column starts
  float4 reg[16];
  uint2 ereg[kPieceLoads];
  uint32_t cp_next = 0, tot_next = 0;
  auto fetch = [&](int64_t ch) {
    if (rows_in && (ch + 1) * kChunk <= n) load_tile<true>(A, lda, m, n, i0, ch * kChunk, lane, reg);
    else load_tile<false>(A, lda, m, n, i0, ch * kChunk, lane, reg);
    const uint2 *eg = reinterpret_cast<const uint2 *>(entries + ch * (int64_t)kEntCap);
#pragma unroll
    for (int j = 0; j < kPieceLoads; ++j) ereg[j] = eg[tid + 64 * kSketchWaves * j];   // < kEntCap
    cp_next = colptr[ch * (kMaxBlock + 1) + lane];
    tot_next = colptr[ch * (kMaxBlock + 1) + kMaxBlock];
  };
  auto stage = [&](int buf) {
    store_tile(tile_lds, lane, reg);
#pragma unroll
    for (int j = 0; j < kPieceLoads; ++j) ents[buf][tid + 64 * kSketchWaves * j] = ereg[j];
  };
  // chunk ch: tile in tile_lds, first piece of its entries in ents[buf]
  auto process = [&](int64_t ch, int buf, uint32_t cp_lane, uint32_t total) {
    const uint32_t p1 = total < (uint32_t)kPiece ? total : (uint32_t)kPiece;
    sketch_piece(acc, ents[buf], tile_bytes, cp_lane, total, 0u, p1, b);
    if (total > (uint32_t)kPiece) {
      // dense column lists: the remaining pieces are staged synchronously
      const uint2 *eg = reinterpret_cast<const uint2 *>(entries + ch * (int64_t)kEntCap);
      for (uint32_t p0 = kPiece; p0 < total; p0 += kPiece) {
        const uint32_t q1 = (total - p0 > (uint32_t)kPiece) ? p0 + kPiece : total;
        __syncthreads();
        for (uint32_t e = p0 + tid; e < q1; e += 64 * kSketchWaves) ents[buf][e - p0] = eg[e];
        __syncthreads();
        sketch_piece(acc, ents[buf], tile_bytes, cp_lane, total, p0, q1, b);
      }
    }
  };

  if (ch_begin < ch_end) {
    fetch(ch_begin);
    stage(0);
    __syncthreads();
    uint32_t cp_cur = cp_next, tot_cur = tot_next;
    int buf = 0;
    for (int64_t ch = ch_begin; ch < ch_end; ++ch) {
      // the last chunk fetches itself again (in bounds, unused): the loads
      // stay unconditional, so no wait lands in front of the LDS work
      fetch(ch + 1 < ch_end ? ch + 1 : ch);
      __builtin_amdgcn_sched_barrier(0);
      process(ch, buf, cp_cur, tot_cur);
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();            // every wave is done with this chunk's tile and entries
      stage(buf ^ 1);
      __syncthreads();
      buf ^= 1;
      cp_cur = cp_next;
      tot_cur = tot_next;
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
    float *o = out + (split * m + row) * (int64_t)kBld;
#pragma unroll
    for (int c = 0; c < kMaxBlock; ++c) o[c] = (c < b) ? acc[c] : 0.0f;
  }
}

// part: nsplit == 1 -> final S (scale, z applied); else partials (nsplit x m x kBld).
void launch_sketch_full(const float *A, int64_t lda, int64_t m, int64_t n, int b,
                        const uint32_t *colptr, const ChunkEntry *entries, float *out,
                        int nsplit, float scale, const float *z, float zc, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  if (nsplit < 1) nsplit = 1;
  if (nsplit > nchunks) nsplit = (int)nchunks;
  const int64_t cps = (nchunks + nsplit - 1) / nsplit;
  nsplit = (int)((nchunks + cps - 1) / cps);
  const bool vec = (lda % 4 == 0) && (lda < (int64_t(1) << 28)) &&
                   ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  const int64_t tiles = (m + 64 * kSketchWaves - 1) / (64 * kSketchWaves);
  const int64_t total = tiles * nsplit;
  dim3 grid((unsigned)total), blk(64 * kSketchWaves);
#define FARPCA_SKETCH_LAUNCH(V, D)                                                              \
  hipLaunchKernelGGL((sketch_kernel<V, D>), grid, blk, 0, st, A, lda, m, n, b, colptr, entries, \
                     out, cps, tiles, total, scale, z, zc)
  if (nsplit == 1) {
    if (vec) FARPCA_SKETCH_LAUNCH(true, true);
    else FARPCA_SKETCH_LAUNCH(false, true);
  } else {
    if (vec) FARPCA_SKETCH_LAUNCH(true, false);
    else FARPCA_SKETCH_LAUNCH(false, false);
  }
#undef FARPCA_SKETCH_LAUNCH
}

// Workgroups of the sketch kernel resident on the current device at once.
static int64_t sketch_slots() {
  static std::mutex mu;
  static std::map<int, int64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void *>(&sketch_kernel<true, false>), 64 * kSketchWaves,
          0) != hipSuccess ||
      per_cu < 1)
    per_cu = 2;
  const int64_t slots = (int64_t)cus * per_cu;
  cache[dev] = slots;
  return slots;
}

// Splits of the chunk range: workgroups in as few rounds of resident
// workgroups as possible, each split >= 4 chunks, partial traffic small next
// to A (time modelled as rounds x (chunks / s) x (1 + 2 s / chunks)).
int sketch_choose_split(int64_t m, int64_t n) {
  const int64_t tiles = (m + 64 * kSketchWaves - 1) / (64 * kSketchWaves);
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  const int64_t slots = sketch_slots();
  int64_t smax = nchunks / 4;
  if (smax > 16) smax = 16;
  int best = 1;
  double best_cost = 0.0;
  for (int64_t sp = 1; sp <= (smax < 1 ? 1 : smax); ++sp) {
    const int64_t rounds = (tiles * sp + slots - 1) / slots;
    const double cost = (double)rounds / (double)sp * (1.0 + 2.0 * (double)sp / (double)nchunks);
    if (sp == 1 || cost < best_cost * (1.0 - 1e-9)) {
      best = (int)sp;
      best_cost = cost;
    }
  }
  return best;
}

}  // namespace farpca_int
