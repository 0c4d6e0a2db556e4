// Sparse sketch S = A * Omega_j for the sparse test matrices (Section 3: the
// cost of A B_j is nnz(B_j) m instead of a dense product).
//
// A (FP32, or BF16 for the precision form: widened exactly to FP32 when the
// tile is stored in LDS, so everything after the load is shared) is streamed
// in chunks of 64 columns.  A workgroup has four waves over one
// block of 128 rows; lane l of every wave owns rows 2 l and 2 l + 1 of the
// block, wave w owns output columns 16 w .. 16 w + 15.  Per chunk
//   1. each wave holds a quarter of the block's 128 x 64 tile of A in
//      registers (16-byte loads, 4 rows x 256 contiguous bytes per
//      instruction; BF16: 8-byte loads, 4 rows x 128 bytes) and stores it transposed into the LDS tile (column-major,
//      130 floats per column: rows 2 l, 2 l + 1 form one aligned 8-byte pair).
//      Tiles are fetched two chunks ahead, so that every wave keeps 16 KB in
//      flight while it works: HBM needs a few hundred KB in flight per CU;
//   2. each wave walks the chunk's column lists of Omega for its 16 output
//      columns (lists staged in LDS once for the workgroup, padded per column
//      to groups of four; every lane reads the same entry: an LDS broadcast),
//      two columns per step, accumulating acc[r][c] += val * tile[j][2 l + r]
//      with one 8-byte tile read per entry for two rows: each A element is
//      read from HBM once and from LDS once per nonzero of its Omega row, and
//      each list entry is read once per 128 rows.
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

constexpr int kRowsWg = 128;              // rows of A per workgroup (2 per lane)
constexpr int kTileStride = kRowsWg + 2;  // floats per LDS column of the staged tile
constexpr int kHalf = kMaxBlock / 4;      // output columns per wave
constexpr int kThreads = 256;
constexpr int kPiece = 768;               // column-list entries staged in LDS at a time
constexpr int kPieceLoads = kPiece / kThreads;   // entries per thread per piece
constexpr int kPair = 2;                  // output columns walked together
static_assert(kPiece % kThreads == 0, "piece must split evenly over the threads");
static_assert(kPiece % kListPad == 0, "pieces hold whole groups");

int sketch_lds_row_stride_bytes() { return kTileStride * 4; }
int sketch_rows_per_wg() { return kRowsWg; }

// Registers of a quarter tile: 4 consecutive columns of A per row and
// instruction, as loaded (FP32: 16 bytes; BF16: 8 bytes, widened to FP32 only
// when the tile is stored, so the loads stay in flight until then).
template <typename T> struct TileRaw;
template <> struct TileRaw<float> { using type = float4; };
template <> struct TileRaw<uint16_t> { using type = uint2; };

// A quarter tile (rows r0 .. r0 + 31) into registers: instruction
// q covers rows r0 + 4 q + lane/16, columns col0 + 4 (lane%16) .. +3.  Rows
// beyond m are clamped to m - 1 (they feed outputs that are never stored) and
// columns beyond n read as zero.  VEC (lda % 4 == 0, A aligned to 4 elements,
// lda < 2^28): one vector load per instruction from a uniform row base plus a
// 32-bit lane offset; a column group that crosses n is read at a clamped
// column inside the row (lda >= n) and then masked.  Otherwise scalar loads.
template <typename T, bool VEC>
__device__ __forceinline__ void load_half(const T *__restrict__ A, int64_t lda, int64_t m,
                                          int64_t n, int64_t r0, int64_t col0, int lane,
                                          typename TileRaw<T>::type (&reg)[8]) {
  const int rsub = lane >> 4;
  const int64_t col = col0 + (lane & 15) * 4;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int64_t rq = (r0 + 4 * q < m) ? r0 + 4 * q : m - 1;
    const int64_t row = (r0 + 4 * q + rsub < m) ? r0 + 4 * q + rsub : m - 1;
    const T *base = A + rq * lda;
    const int32_t roff = (int32_t)(row - rq) * (int32_t)lda;
    if (VEC) {
      const int64_t cc = col < lda - 4 ? col : lda - 4;
      bool ok[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) ok[t] = col + t < n && cc == col;
      if constexpr (sizeof(T) == 4) {
        const float4 u = *reinterpret_cast<const float4 *>(base + (roff + (int32_t)cc));
        reg[q] = make_float4(ok[0] ? u.x : 0.0f, ok[1] ? u.y : 0.0f, ok[2] ? u.z : 0.0f,
                             ok[3] ? u.w : 0.0f);
      } else {
        const uint2 u = *reinterpret_cast<const uint2 *>(base + (roff + (int32_t)cc));
        const uint32_t m0 = (ok[0] ? 0x0000FFFFu : 0u) | (ok[1] ? 0xFFFF0000u : 0u);
        const uint32_t m1 = (ok[2] ? 0x0000FFFFu : 0u) | (ok[3] ? 0xFFFF0000u : 0u);
        reg[q] = make_uint2(u.x & m0, u.y & m1);
      }
    } else {
      T v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t c = col + t < n ? col + t : n - 1;
        const T u = base[roff + (int32_t)c];
        v[t] = (col + t < n) ? u : T(0);
      }
      if constexpr (sizeof(T) == 4) {
        reg[q] = make_float4(v[0], v[1], v[2], v[3]);
      } else {
        reg[q] = make_uint2((uint32_t)v[0] | ((uint32_t)v[1] << 16),
                            (uint32_t)v[2] | ((uint32_t)v[3] << 16));
      }
    }
  }
}

__device__ __forceinline__ float4 widen(const float4 &v) { return v; }
// BF16 bit patterns (low half first) to FP32: exact.
__device__ __forceinline__ float4 widen(const uint2 &v) {
  return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xFFFF0000u),
                     __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xFFFF0000u));
}

// Store a quarter tile transposed: tile[col][row] with row = 32 w + 4 q + lane/16.
template <typename R>
__device__ __forceinline__ void store_half(float *tile, int w, int lane, const R (&reg)[8]) {
  const int rsub = lane >> 4;
  const int c4 = (lane & 15) * 4;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int row = 32 * w + 4 * q + rsub;
    const float4 v = widen(reg[q]);
    tile[(c4 + 0) * kTileStride + row] = v.x;
    tile[(c4 + 1) * kTileStride + row] = v.y;
    tile[(c4 + 2) * kTileStride + row] = v.z;
    tile[(c4 + 3) * kTileStride + row] = v.w;
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
// kPiece + 3] zero.  Adds the lists of output columns c_base .. c_base + 15
// into acc (the lane's two rows), kPair columns per step.  cp0 / cp1 (lane c): start / end of
// column c.
__device__ __forceinline__ void sketch_piece(float (&acc)[2][kHalf], const uint2 *E,
                                             const char *tile_bytes, uint32_t cp0, uint32_t cp1,
                                             int c_base, uint32_t p0, uint32_t p1, int b) {
#pragma unroll
  for (int cq = 0; cq < kHalf; cq += kPair) {
    if (c_base + cq < b) {
      uint32_t lo[kPair], len[kPair];
      uint32_t kmax = 0;
#pragma unroll
      for (int i = 0; i < kPair; ++i) {
        const int c = c_base + cq + i;
        const uint32_t c0 = __builtin_amdgcn_readlane(cp0, c);
        const uint32_t c1 = __builtin_amdgcn_readlane(cp1, c);
        const uint32_t l0 = c0 > p0 ? c0 : p0;
        const uint32_t h0 = c1 < p1 ? c1 : p1;
        len[i] = h0 > l0 ? h0 - l0 : 0u;      // a multiple of kListPad
        lo[i] = h0 > l0 ? l0 - p0 : 0u;
        kmax = len[i] > kmax ? len[i] : kmax;
      }
      if (kmax == 0) continue;
      float a0[kPair], a1[kPair];
#pragma unroll
      for (int i = 0; i < kPair; ++i) { a0[i] = acc[0][cq + i]; a1[i] = acc[1][cq + i]; }
      // entries of step k (past a column's end: the zero group)
      auto read_entries = [&](uint32_t k, uint2 (&q)[kPair][kListPad]) {
#pragma unroll
        for (int i = 0; i < kPair; ++i) {
          const uint32_t base = (k < len[i]) ? lo[i] + k : (uint32_t)kPiece;   // + 3 < kPiece + 4
#pragma unroll
          for (int u = 0; u < kListPad; ++u) q[i][u] = E[base + u];
        }
      };
      auto accumulate = [&](const uint2 (&q)[kPair][kListPad]) {
        float2 x[kPair][kListPad];
#pragma unroll
        for (int i = 0; i < kPair; ++i)
#pragma unroll
          for (int u = 0; u < kListPad; ++u)
            x[i][u] = *reinterpret_cast<const float2 *>(tile_bytes + q[i][u].x);
#pragma unroll
        for (int i = 0; i < kPair; ++i)
#pragma unroll
          for (int u = 0; u < kListPad; ++u) {
            const float v = __uint_as_float(q[i][u].y);
            a0[i] = fmaf(v, x[i][u].x, a0[i]);
            a1[i] = fmaf(v, x[i][u].y, a1[i]);
          }
      };
      for (uint32_t k = 0; k < kmax; k += kListPad) {
        uint2 qa[kPair][kListPad];
        read_entries(k, qa);
        accumulate(qa);
      }
#pragma unroll
      for (int i = 0; i < kPair; ++i) { acc[0][cq + i] = a0[i]; acc[1][cq + i] = a1[i]; }
    }
  }
}

template <typename T, bool VEC, bool DIRECT>
__global__ __launch_bounds__(kThreads) void sketch_kernel(
    const T *__restrict__ A, int64_t lda, int64_t m, int64_t n, int b,
    const uint32_t *__restrict__ colptr, const ChunkEntry *__restrict__ entries,
    float *__restrict__ out, int64_t chunks_per_split, int64_t tiles, int64_t total_wg,
    float scale, const float *__restrict__ z, float zc) {
  __shared__ float tile_lds[kChunk * kTileStride];
  __shared__ uint2 ents[2][kPiece + kListPad];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int64_t L = sketch_xcd_remap(blockIdx.x, total_wg);
  const int64_t tile = L % tiles, split = L / tiles;
  const int64_t i0 = tile * kRowsWg;
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  const int64_t ch_begin = split * chunks_per_split;
  int64_t ch_end = ch_begin + chunks_per_split;
  if (ch_end > nchunks) ch_end = nchunks;
  const char *tile_bytes = reinterpret_cast<const char *>(tile_lds) + lane * 8;
  const int c_base = kHalf * wave;

  if (tid < 2 * kListPad) ents[tid / kListPad][kPiece + tid % kListPad] = make_uint2(0u, 0u);

  float acc[2][kHalf];
#pragma unroll
  for (int c = 0; c < kHalf; ++c) { acc[0][c] = 0.0f; acc[1][c] = 0.0f; }

  // quarter tiles of chunks ch + 1 (one set) and ch + 2 (the other) in flight
  using Raw = typename TileRaw<T>::type;
  Raw s0[8], s1[8];
  auto fetch_tile = [&](int64_t ch, Raw (&reg)[8]) {
    load_half<T, VEC>(A, lda, m, n, i0 + 32 * wave, ch * kChunk, lane, reg);
  };
  // first piece of a chunk's entries and its column bounds (one chunk ahead)
  uint2 ereg[kPieceLoads];
  uint32_t cp0_next = 0, cp1_next = 0;
  auto fetch_lists = [&](int64_t ch) {
    const uint2 *eg = reinterpret_cast<const uint2 *>(entries + ch * (int64_t)kEntCap);
#pragma unroll
    for (int j = 0; j < kPieceLoads; ++j) ereg[j] = eg[tid + kThreads * j];   // < kEntCap
    cp0_next = colptr[ch * (kMaxBlock + 1) + lane];
    cp1_next = colptr[ch * (kMaxBlock + 1) + lane + 1];
  };
  auto stage_lists = [&](int buf) {
#pragma unroll
    for (int j = 0; j < kPieceLoads; ++j) ents[buf][tid + kThreads * j] = ereg[j];
  };
  // chunk ch: tile in tile_lds, first piece of its entries in ents[buf]
  auto process = [&](int64_t ch, int buf, uint32_t cp0, uint32_t cp1) {
    const uint32_t total = __builtin_amdgcn_readlane(cp1, kMaxBlock - 1);
    const uint32_t p1 = total < (uint32_t)kPiece ? total : (uint32_t)kPiece;
    sketch_piece(acc, ents[buf], tile_bytes, cp0, cp1, c_base, 0u, p1, b);
    if (total > (uint32_t)kPiece) {
      // dense column lists: the remaining pieces are staged synchronously
      const uint2 *eg = reinterpret_cast<const uint2 *>(entries + ch * (int64_t)kEntCap);
      for (uint32_t p0 = kPiece; p0 < total; p0 += kPiece) {
        const uint32_t q1 = (total - p0 > (uint32_t)kPiece) ? p0 + kPiece : total;
        __syncthreads();
        for (uint32_t e = p0 + tid; e < q1; e += kThreads) ents[buf][e - p0] = eg[e];
        __syncthreads();
        sketch_piece(acc, ents[buf], tile_bytes, cp0, cp1, c_base, p0, q1, b);
      }
    }
  };
  // one chunk: fetch ahead (lists of ch + 1 first, then the tile of ch + 2, so
  // the wait before staging ch + 1 leaves the newest tile loads in flight),
  // walk ch, stage ch + 1 from `nxt`; `far` receives ch + 2
  auto iterate = [&](int64_t ch, int buf, uint32_t &cp0, uint32_t &cp1, Raw (&nxt)[8],
                     Raw (&far)[8]) {
    const int64_t c1 = ch + 1 < ch_end ? ch + 1 : ch;      // clamped: in bounds, unused
    const int64_t c2 = ch + 2 < ch_end ? ch + 2 : ch;
    fetch_lists(c1);
    fetch_tile(c2, far);
    __builtin_amdgcn_sched_barrier(0);
    process(ch, buf, cp0, cp1);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();                 // every wave is done with this chunk's tile and lists
    if (ch + 1 < ch_end) {
      store_half(tile_lds, wave, lane, nxt);
      stage_lists(buf ^ 1);
    }
    __syncthreads();
    cp0 = cp0_next;
    cp1 = cp1_next;
  };

  if (ch_begin < ch_end) {
    fetch_lists(ch_begin);
    fetch_tile(ch_begin, s0);
    fetch_tile(ch_begin + 1 < ch_end ? ch_begin + 1 : ch_begin, s1);
    store_half(tile_lds, wave, lane, s0);
    stage_lists(0);
    __syncthreads();
    uint32_t cp0 = cp0_next, cp1 = cp1_next;
    // s1 holds chunk ch + 1 at even steps, s0 at odd steps
    int buf = 0;
    for (int64_t ch = ch_begin; ch < ch_end; ++ch) {
      iterate(ch, buf, cp0, cp1, s1, s0);
#pragma unroll
      for (int q = 0; q < 8; ++q) s1[q] = s0[q];
      buf ^= 1;
    }
  }

#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int64_t row = i0 + 2 * lane + r;
    if (row >= m) continue;
    if (DIRECT) {
      float *o = out + row * (int64_t)kBld + c_base;
      const float zr = z ? zc * z[row] : 0.0f;
#pragma unroll
      for (int c = 0; c < kHalf; ++c) o[c] = (c_base + c < b) ? fmaf(scale, acc[r][c], zr) : 0.0f;
    } else {
      float *o = out + (split * m + row) * (int64_t)kBld + c_base;
#pragma unroll
      for (int c = 0; c < kHalf; ++c) o[c] = (c_base + c < b) ? acc[r][c] : 0.0f;
    }
  }
}

template <typename T>
static void launch_sketch_t(const T *A, int64_t lda, int64_t m, int64_t n, int b,
                            const uint32_t *colptr, const ChunkEntry *entries, float *out,
                            int nsplit, float scale, const float *z, float zc, hipStream_t st) {
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  if (nsplit < 1) nsplit = 1;
  if (nsplit > nchunks) nsplit = (int)nchunks;
  const int64_t cps = (nchunks + nsplit - 1) / nsplit;
  nsplit = (int)((nchunks + cps - 1) / cps);
  const bool vec = (lda % 4 == 0) && (lda < (int64_t(1) << 28)) &&
                   ((reinterpret_cast<uintptr_t>(A) & (4 * sizeof(T) - 1)) == 0);
  const int64_t tiles = (m + kRowsWg - 1) / kRowsWg;
  const int64_t total = tiles * nsplit;
  dim3 grid((unsigned)total), blk(kThreads);
#define FARPCA_SKETCH_LAUNCH(V, D)                                                                 \
  hipLaunchKernelGGL((sketch_kernel<T, V, D>), grid, blk, 0, st, A, lda, m, n, b, colptr, entries, \
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

// part: nsplit == 1 -> final S (scale, z applied); else partials (nsplit x m x kBld).
void launch_sketch_full(const void *A, bool bf16, int64_t lda, int64_t m, int64_t n, int b,
                        const uint32_t *colptr, const ChunkEntry *entries, float *out,
                        int nsplit, float scale, const float *z, float zc, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  if (bf16)
    launch_sketch_t(static_cast<const uint16_t *>(A), lda, m, n, b, colptr, entries, out, nsplit,
                    scale, z, zc, st);
  else
    launch_sketch_t(static_cast<const float *>(A), lda, m, n, b, colptr, entries, out, nsplit,
                    scale, z, zc, st);
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
          &per_cu, reinterpret_cast<const void *>(&sketch_kernel<float, true, false>), kThreads, 0) !=
          hipSuccess ||
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
  const int64_t tiles = (m + kRowsWg - 1) / kRowsWg;
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
