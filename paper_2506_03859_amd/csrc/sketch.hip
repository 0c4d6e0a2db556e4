// Sparse sketch S = A * Omega_j for the sparse test matrices (Section 3: the
// cost of A B_j is nnz(B_j) m instead of a dense product).
//
// A (FP32, or BF16 for the precision form: widened exactly to FP32 when the
// tile is stored in LDS, so everything after the load is shared) is streamed
// in chunks of 64 columns.  A workgroup has eight waves over one block of 256
// rows; lane l of every wave owns rows 4 l .. 4 l + 3 of the block, wave w owns
// output columns 8 w .. 8 w + 7.  Per chunk
//   1. each wave loads an eighth of the block's 256 x 64 tile of A into
//      registers (16-byte loads, 4 rows x 256 contiguous bytes per
//      instruction; BF16: 8-byte loads, 4 rows x 128 bytes) one chunk ahead,
//      and stores it transposed into the LDS tile (column-major, 260 floats
//      per column), four rows per 16-byte store: the lanes of a store cycle
//      cover every bank once;
//   2. each wave walks the chunk's column lists of Omega for its 8 output
//      columns, accumulating acc[r][c] += val * tile[k][4 l + r] with one
//      16-byte tile read per entry for four rows.  The lists are loaded one
//      chunk ahead into registers (lane j holds entries j and 64 + j of the
//      wave's stream) and each entry is broadcast to the wave with readlane,
//      so the LDS serves only the tile: each A element is read from HBM once
//      and from LDS once per nonzero of its Omega row.
// The lists of the wave's columns are contiguous (one stream) and each is
// padded to whole groups of four with zero entries (0 * finite = +0, an exact
// no-op).  Each column's sum runs in list order, so results are bitwise
// repeatable; the +-1 values of the sign sketches are added exactly (no
// scaling until the final multiply).  Chunks are split into consecutive groups
// (K splits) to fill the GPU; the partial sums are reduced in split order by
// reduce_partials.
#include <map>
#include <mutex>

#include "internal.h"

namespace farpca_int {

constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kRowsLane = 4;                 // rows per lane (one 16-byte tile read)
constexpr int kRowsWg = 64 * kRowsLane;      // rows of A per workgroup
constexpr int kRowsWave = kRowsWg / kWaves;  // rows each wave loads and stores
constexpr int kTileStride = kRowsWg + 4;     // floats per LDS column of the staged tile
constexpr int kCols = kMaxBlock / kWaves;    // output columns per wave
constexpr int kWin = 128;                    // list entries a wave holds in registers
static_assert(kTileStride % 32 == 4, "column stride 4 mod 32 keeps the 16-byte stores conflict-free");
static_assert(kRowsWave == 32, "a wave loads 8 instructions of 4 rows");
static_assert(kEntCap >= kChunk * kMaxBlock + (kListPad - 1) * kMaxBlock + kWin,
              "a window read past the last list stays inside the chunk's region");

int sketch_lds_row_stride_bytes() { return kTileStride * 4; }
int sketch_rows_per_wg() { return kRowsWg; }

// Registers of one wave's share of a tile: 4 consecutive columns of A per row
// and instruction, as loaded (FP32: 16 bytes; BF16: 8 bytes, widened to FP32
// only when the tile is stored, so the loads stay in flight until then).
template <typename T> struct TileRaw;
template <> struct TileRaw<float> { using type = float4; };
template <> struct TileRaw<uint16_t> { using type = uint2; };

// Rows r0 .. r0 + 31 of a chunk into registers.  Lane l serves the row quad
// p = l % 4 and the column group l / 4: instruction 4 g + h covers rows
// r0 + 16 g + 4 p + h, columns col0 + 4 (l / 4) .. +3 (4 rows x 64 columns per
// instruction), so that a lane holds rows 4 p .. 4 p + 3 of the same columns
// for the 16-byte store.  ROWS_FULL: all 32 rows exist.  Otherwise a lane
// whose row is beyond m reads the instruction's first row instead, clamped to
// m - 1 (it feeds outputs that are never stored).  VEC (lda % 4 == 0, A
// aligned to 4 elements, lda < 2^26): one vector load per instruction from a
// uniform base (row and chunk) plus a 32-bit lane byte offset; a column group
// past n is read at a clamped column inside the row (lda >= n) and masked
// when the tile is stored, so no load waits early.  Otherwise element loads
// that read columns past n as zero.
template <typename T, bool VEC, bool ROWS_FULL>
__device__ __forceinline__ void load_share(const T *__restrict__ A, int64_t lda, int64_t m,
                                           int64_t n, int64_t r0, int64_t col0, int lane,
                                           typename TileRaw<T>::type (&reg)[8]) {
  using Raw = typename TileRaw<T>::type;
  const int rsub = 4 * (lane & 3);
  const int64_t col = col0 + (lane >> 2) * 4;
  if (VEC) {
    const int64_t cc = col < lda - 4 ? col : lda - 4;
    const uint32_t lcol = (uint32_t)(cc - col0) * (uint32_t)sizeof(T);
    const uint32_t lrow = (uint32_t)rsub * (uint32_t)lda * (uint32_t)sizeof(T);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t rb = r0 + 16 * (q >> 2) + (q & 3);       // the instruction's first row
      const int64_t rq = (ROWS_FULL || rb < m) ? rb : m - 1;
      const char *base = reinterpret_cast<const char *>(A + rq * lda + col0);
      const uint32_t roff = (ROWS_FULL || rb + rsub < m) ? lrow : 0u;
      reg[q] = *reinterpret_cast<const Raw *>(base + (roff + lcol));
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t rb = r0 + 16 * (q >> 2) + (q & 3);
      const int64_t row = (rb + rsub < m) ? rb + rsub : (rb < m ? rb : m - 1);
      const T *rp = A + row * lda;
      T v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t c = col + t < n ? col + t : n - 1;
        const T u = rp[c];
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

// Store a wave's share transposed, four rows per 16-byte store:
// tile[col][row .. row + 3] with row = 32 w + 16 g + 4 (lane % 4), col =
// 4 (lane / 4) + t.  With the column stride 4 mod 32 (in floats) the 8 lanes
// of a store cycle hit 8 distinct 16-byte bank groups (all 32 banks; also all
// 64 for 16 lanes).  In the chunk that crosses n, columns past n are stored
// as zero.
template <typename R>
__device__ __forceinline__ void store_share(float *tile, int w, int lane, const R (&reg)[8],
                                            int64_t col0, int64_t n) {
  const int rsub = 4 * (lane & 3);
  const int c4 = (lane >> 2) * 4;
  const bool full = col0 + kChunk <= n;                      // uniform
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const int row = kRowsWave * w + 16 * g + rsub;
    float4 v[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) v[h] = widen(reg[4 * g + h]);
    float4 c[4] = {make_float4(v[0].x, v[1].x, v[2].x, v[3].x),
                   make_float4(v[0].y, v[1].y, v[2].y, v[3].y),
                   make_float4(v[0].z, v[1].z, v[2].z, v[3].z),
                   make_float4(v[0].w, v[1].w, v[2].w, v[3].w)};
    if (!full) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const bool ok = col0 + c4 + t < n;
        c[t].x = ok ? c[t].x : 0.0f;
        c[t].y = ok ? c[t].y : 0.0f;
        c[t].z = ok ? c[t].z : 0.0f;
        c[t].w = ok ? c[t].w : 0.0f;
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) *reinterpret_cast<float4 *>(tile + (c4 + t) * kTileStride + row) = c[t];
  }
}

// Logical workgroup id (see gemm.hip): XCD x runs physical ids 8 j + x; the
// regrouping gives it a contiguous range of logical ids, i.e. one K split.
__device__ __forceinline__ int64_t sketch_xcd_remap(int64_t g, int64_t T) {
  const int64_t T8 = T & ~int64_t(7);
  if (g >= T8) return g;
  return (g & 7) * (T8 >> 3) + (g >> 3);
}

// A window of a wave's list stream: lane j holds entries base + j (lo) and
// base + 64 + j (hi).  Reads past the stream stay inside the chunk's region
// (the 128 spare slots after the lists).
struct EntWindow { uint2 lo, hi; };

__device__ __forceinline__ EntWindow load_window(const uint2 *E, uint32_t base, int lane) {
  return EntWindow{E[base + lane], E[base + 64 + lane]};
}

// A group of four entries as one 32-byte scalar load: lists start at
// multiples of four entries and the chunk regions are 32-byte aligned.  The
// lists are not written while the sketch runs, so they are read through the
// constant address space (scalar loads with a uniform address).
typedef uint32_t EntGroup __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(4))) const EntGroup ConstGroup;

// One chunk for the wave's output columns c_base .. c_base + 7 (those < b).
// bound[i] = start of column c_base + i's list (bound[kCols] = end of the
// stream); win holds the stream from bound[0] on, loaded a chunk ahead.  A
// group of four entries never straddles the window's halves (lists start at
// multiples of four); a group past the window (only dense lists get there)
// is read with a scalar load.  Each column adds its entries in list order.
// The columns are a compile-time recursion, so that every accumulator index
// is a constant (the accumulators stay in registers).
template <int CQ>
struct ChunkWalk {
  static __device__ __forceinline__ void run(float (&acc)[kRowsLane][kCols], ConstGroup *G,
                                             const uint32_t (&bound)[kCols + 1],
                                             const EntWindow &win, const char *tile_bytes,
                                             int c_base, int b, uint32_t e) {
    if (c_base + CQ >= b) return;
    const uint32_t hi = bound[CQ + 1];
    float a0 = acc[0][CQ], a1 = acc[1][CQ], a2 = acc[2][CQ], a3 = acc[3][CQ];
    for (; e < hi; e += 4) {
      uint32_t off[4], val[4];
      const uint32_t rel = e - bound[0];
      if (rel < 64u) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          off[u] = __builtin_amdgcn_readlane(win.lo.x, rel + u);
          val[u] = __builtin_amdgcn_readlane(win.lo.y, rel + u);
        }
      } else if (rel < (uint32_t)kWin) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          off[u] = __builtin_amdgcn_readlane(win.hi.x, rel - 64u + u);
          val[u] = __builtin_amdgcn_readlane(win.hi.y, rel - 64u + u);
        }
      } else {
        const EntGroup g = G[e / 4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          off[u] = g[2 * u];
          val[u] = g[2 * u + 1];
        }
      }
      float4 x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = *reinterpret_cast<const float4 *>(tile_bytes + off[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float v = __uint_as_float(val[u]);
        a0 = fmaf(v, x[u].x, a0);
        a1 = fmaf(v, x[u].y, a1);
        a2 = fmaf(v, x[u].z, a2);
        a3 = fmaf(v, x[u].w, a3);
      }
    }
    acc[0][CQ] = a0;
    acc[1][CQ] = a1;
    acc[2][CQ] = a2;
    acc[3][CQ] = a3;
    ChunkWalk<CQ + 1>::run(acc, G, bound, win, tile_bytes, c_base, b, hi);
  }
};
template <>
struct ChunkWalk<kCols> {
  static __device__ __forceinline__ void run(float (&)[kRowsLane][kCols], ConstGroup *,
                                             const uint32_t (&)[kCols + 1], const EntWindow &,
                                             const char *, int, int, uint32_t) {}
};

// The chunk range [ch_begin, ch_end) of one row block (rows i0 .. i0 + 255;
// ROWS_FULL: all inside m) into acc.
template <typename T, bool VEC, bool ROWS_FULL>
__device__ __forceinline__ void sketch_rows(float (&acc)[kRowsLane][kCols], float *tile_lds,
                                            const T *__restrict__ A, int64_t lda, int64_t m,
                                            int64_t n, int b, const uint32_t *__restrict__ colptr,
                                            const uint2 *ent, int64_t i0, int64_t ch_begin,
                                            int64_t ch_end, int wave, int lane) {
  const char *tile_bytes = reinterpret_cast<const char *>(tile_lds) + lane * 16;
  const int c_base = kCols * wave;
  const int64_t r0 = i0 + kRowsWave * wave;
  using Raw = typename TileRaw<T>::type;
  Raw nxt[8];
  // column starts c_base .. c_base + kCols of chunk ch: lane i <= kCols holds
  // entry c_base + i (the others repeat the last)
  auto load_bounds = [&](int64_t ch) {
    const int i = lane < kCols ? lane : kCols;
    return colptr[ch * (kMaxBlock + 1) + c_base + i];
  };
  auto chunk_entries = [&](int64_t ch) { return ent + ch * (int64_t)kEntCap; };

  uint32_t bv = load_bounds(ch_begin);
  uint32_t bound[kCols + 1];
#pragma unroll
  for (int i = 0; i <= kCols; ++i) bound[i] = __builtin_amdgcn_readlane(bv, i);
  EntWindow win = load_window(chunk_entries(ch_begin), bound[0], lane);
  uint32_t bv_next = load_bounds(ch_begin + 1 < ch_end ? ch_begin + 1 : ch_begin);
  load_share<T, VEC, ROWS_FULL>(A, lda, m, n, r0, ch_begin * kChunk, lane, nxt);
  store_share(tile_lds, wave, lane, nxt, ch_begin * kChunk, n);
  __syncthreads();
  for (int64_t ch = ch_begin; ch < ch_end; ++ch) {
    // ahead: lists of ch + 1 (their bounds arrived last step), bounds of
    // ch + 2, then the tile of ch + 1, in this order: the wait before the tile
    // store then also covers the lists and bounds
    const int64_t c1 = ch + 1 < ch_end ? ch + 1 : ch;      // clamped: in bounds, unused
    const int64_t c2 = ch + 2 < ch_end ? ch + 2 : c1;
    uint32_t bound_next[kCols + 1];
#pragma unroll
    for (int i = 0; i <= kCols; ++i) bound_next[i] = __builtin_amdgcn_readlane(bv_next, i);
    const EntWindow win_next = load_window(chunk_entries(c1), bound_next[0], lane);
    const uint32_t bv_far = load_bounds(c2);
    load_share<T, VEC, ROWS_FULL>(A, lda, m, n, r0, c1 * kChunk, lane, nxt);
    __builtin_amdgcn_sched_barrier(0);
    ChunkWalk<0>::run(acc, (ConstGroup *)(uintptr_t)chunk_entries(ch), bound, win, tile_bytes,
                      c_base, b, bound[0]);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();               // every wave is done with this chunk's tile
    if (ch + 1 < ch_end) store_share(tile_lds, wave, lane, nxt, c1 * kChunk, n);
    __syncthreads();
#pragma unroll
    for (int i = 0; i <= kCols; ++i) bound[i] = bound_next[i];
    win = win_next;
    bv_next = bv_far;
  }
}

// Two workgroups per CU (LDS: 2 x 65 KB): 16 waves, 4 per SIMD, so at most
// 128 registers per lane.
template <typename T, bool VEC, bool DIRECT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void sketch_kernel(
    const T *__restrict__ A, int64_t lda, int64_t m, int64_t n, int b,
    const uint32_t *__restrict__ colptr, const ChunkEntry *__restrict__ entries,
    float *__restrict__ out, int64_t chunks_per_split, int64_t tiles, int64_t total_wg,
    float scale, const float *__restrict__ z, float zc) {
  __shared__ float tile_lds[kChunk * kTileStride];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);    // uniform
  const int64_t L = sketch_xcd_remap(blockIdx.x, total_wg);
  const int64_t tile = L % tiles, split = L / tiles;
  const int64_t i0 = tile * kRowsWg;
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  const int64_t ch_begin = split * chunks_per_split;
  int64_t ch_end = ch_begin + chunks_per_split;
  if (ch_end > nchunks) ch_end = nchunks;
  const int c_base = kCols * wave;
  const uint2 *ent = reinterpret_cast<const uint2 *>(entries);

  float acc[kRowsLane][kCols];
#pragma unroll
  for (int c = 0; c < kCols; ++c)
#pragma unroll
    for (int r = 0; r < kRowsLane; ++r) acc[r][c] = 0.0f;
  if (ch_begin < ch_end) {
    if (i0 + kRowsWg <= m)
      sketch_rows<T, VEC, true>(acc, tile_lds, A, lda, m, n, b, colptr, ent, i0, ch_begin, ch_end,
                                wave, lane);
    else
      sketch_rows<T, VEC, false>(acc, tile_lds, A, lda, m, n, b, colptr, ent, i0, ch_begin, ch_end,
                                 wave, lane);
  }

#pragma unroll
  for (int r = 0; r < kRowsLane; ++r) {
    const int64_t row = i0 + kRowsLane * lane + r;
    if (row >= m) continue;
    if (DIRECT) {
      float *o = out + row * (int64_t)kBld + c_base;
      const float zr = z ? zc * z[row] : 0.0f;
#pragma unroll
      for (int c = 0; c < kCols; ++c) o[c] = (c_base + c < b) ? fmaf(scale, acc[r][c], zr) : 0.0f;
    } else {
      float *o = out + (split * m + row) * (int64_t)kBld + c_base;
#pragma unroll
      for (int c = 0; c < kCols; ++c) o[c] = (c_base + c < b) ? acc[r][c] : 0.0f;
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
  const bool vec = (lda % 4 == 0) && (lda < (int64_t(1) << 26)) &&
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
