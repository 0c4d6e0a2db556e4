// A stored column-major (A^T row-major: row k of the stored matrix is column
// k of A, m contiguous floats).  In this layout the sparse sketch is a gather
// of whole columns of A, so it reads only the columns that Omega_j touches:
// nnz(Omega_j) m elements instead of m n (Section 3, the cost of A B_j; the
// reason the paper's sparse test matrices pay off for p near 1e-3).
//
//   flatten_lists_kernel  per-chunk column lists of omega_kernel (generated
//                         with row offsets inside the chunk) -> one list per
//                         column of Omega_j over all n rows, ascending row,
//                         padding entries dropped
//   sketch_cols_kernel    S[i][c] = scale * sum_e val_e A[i][k_e] + zc z[i]
//   colsum_kernel         row sums of A (column sums of the stored matrix) in
//                         FP64, for the standardized Bernoulli correction
//
// A wave owns 256 consecutive rows of A (4 per lane, one 16-byte load per
// entry: 1 KB contiguous per wave) and 4 output columns; it walks the lists
// of its columns in order, 8 entries (8 independent loads) at a time.  Each
// column's sum runs in list order, the same order the row-major sketch adds
// the column's entries in.
#include "internal.h"

namespace farpca_int {

constexpr int kGatherCols = 4;                          // output columns per wave
constexpr int kGatherRows = 256;                        // rows of A per wave
constexpr int kGatherGroups = kMaxBlock / kGatherCols;  // column groups per row tile
constexpr int kGatherUnroll = 8;                        // entries in flight per wave

// ---------------------------------------------------------------- flatten
// One wave per column c < b.  Lane t takes chunk g + t of each group of 64
// chunks: its count of real entries (value != 0: the zero-valued padding of
// the chunk lists is dropped, which only removes additions of +0), an
// exclusive prefix over the lanes, then the entries at their positions.
__global__ __launch_bounds__(64) void flatten_lists_kernel(const uint32_t *__restrict__ colptr,
                                                           const ChunkEntry *__restrict__ entries,
                                                           int64_t nchunks, int64_t n,
                                                           ChunkEntry *__restrict__ flat,
                                                           uint32_t *__restrict__ colcnt) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  ChunkEntry *out = flat + (int64_t)c * n;
  uint32_t base = 0;
  for (int64_t g = 0; g < nchunks; g += 64) {
    const int64_t ch = g + lane;
    uint32_t s = 0, e = 0, cnt = 0;
    const ChunkEntry *ent = entries + (ch < nchunks ? ch : 0) * (int64_t)kEntCap;
    if (ch < nchunks) {
      const uint32_t *cp = colptr + ch * (kMaxBlock + 1);
      s = cp[c];
      e = cp[c + 1];
      for (uint32_t q = s; q < e; ++q) cnt += (ent[q].val != 0.0f) ? 1u : 0u;
    }
    uint32_t incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    uint32_t pos = base + incl - cnt;
    for (uint32_t q = s; q < e; ++q) {
      const ChunkEntry x = ent[q];
      if (x.val != 0.0f) {
        ChunkEntry y;
        y.lds_off = (uint32_t)(ch * kChunk) + x.lds_off;   // row of Omega_j = column of A
        y.val = x.val;
        out[pos++] = y;
      }
    }
    base += __shfl(incl, 63, 64);
  }
  if (lane == 0) colcnt[c] = base;
}

void launch_flatten_lists(const uint32_t *colptr, const ChunkEntry *entries, int64_t n, int b,
                          ChunkEntry *flat, uint32_t *colcnt, hipStream_t st) {
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  hipLaunchKernelGGL(flatten_lists_kernel, dim3((unsigned)b), dim3(64), 0, st, colptr, entries,
                     nchunks, n, flat, colcnt);
}

// ---------------------------------------------------------------- gather
// The lists are not written while the kernel runs: read them through the
// constant address space (scalar loads; the entry index is wave-uniform).
typedef uint32_t EntPair __attribute__((ext_vector_type(2)));   // (row, value bits)
typedef __attribute__((address_space(4))) const EntPair ConstEnt;
typedef __attribute__((address_space(4))) const uint32_t ConstU32;

// Rows i0 .. i0 + 3 of column k of A: one 16-byte load when the wave's rows
// all lie inside A and the rows are 16-byte aligned (FULL), else guarded
// scalar loads (zero past row m).
template <bool FULL>
__device__ __forceinline__ float4 col_piece(const float *__restrict__ A, int64_t lda, int64_t m,
                                            uint32_t k, int64_t i0) {
  const float *p = A + (int64_t)k * lda + i0;
  if (FULL) return *reinterpret_cast<const float4 *>(p);
  float v[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) v[r] = (i0 + r < m) ? p[r] : 0.0f;
  return make_float4(v[0], v[1], v[2], v[3]);
}

__device__ __forceinline__ void fma4(float4 &acc, float v, const float4 &a) {
  acc.x = fmaf(v, a.x, acc.x);
  acc.y = fmaf(v, a.y, acc.y);
  acc.z = fmaf(v, a.z, acc.z);
  acc.w = fmaf(v, a.w, acc.w);
}

// The wave's 4 columns (those < b), each summed in list order.
template <bool FULL>
__device__ __forceinline__ void gather_cols(float4 (&acc)[kGatherCols], const float *__restrict__ A,
                                            int64_t lda, int64_t m, int64_t n, int b, int cg,
                                            const ChunkEntry *flat, const uint32_t *colcnt,
                                            int64_t i0) {
#pragma unroll
  for (int cc = 0; cc < kGatherCols; ++cc) {
    const int c = cg * kGatherCols + cc;
    const uint32_t cnt = (c < b) ? *((ConstU32 *)(uintptr_t)(colcnt + c)) : 0u;
    ConstEnt *L = (ConstEnt *)(uintptr_t)(flat + (int64_t)c * n);
    float4 a = acc[cc];
    // groups of kGatherUnroll entries, the last one partial: its missing
    // entries become (column 0, value 0), a load of valid memory that is not
    // used and an addition skipped (the condition is wave-uniform), so every
    // group keeps its loads in flight together
    for (uint32_t e = 0; e < cnt; e += kGatherUnroll) {
      EntPair x[kGatherUnroll];
      float4 v[kGatherUnroll];
#pragma unroll
      for (int u = 0; u < kGatherUnroll; ++u) {
        x[u] = EntPair{0u, 0u};
        if (e + u < cnt) x[u] = L[e + u];
      }
#pragma unroll
      for (int u = 0; u < kGatherUnroll; ++u) v[u] = col_piece<FULL>(A, lda, m, x[u].x, i0);
#pragma unroll
      for (int u = 0; u < kGatherUnroll; ++u)
        if (e + u < cnt) fma4(a, __uint_as_float(x[u].y), v[u]);
    }
    acc[cc] = a;
  }
}

template <bool VEC>
__global__ __launch_bounds__(256) void sketch_cols_kernel(const float *__restrict__ A, int64_t lda,
                                                          int64_t m, int64_t n, int b,
                                                          const ChunkEntry *__restrict__ flat,
                                                          const uint32_t *__restrict__ colcnt,
                                                          float *__restrict__ out, int64_t nwaves,
                                                          float scale, const float *__restrict__ z,
                                                          float zc) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t wid = (int64_t)blockIdx.x * 4 + wave;
  if (wid >= nwaves) return;
  const int64_t tile = wid / kGatherGroups;
  const int cg = (int)(wid % kGatherGroups);
  const int64_t i0 = tile * kGatherRows + 4 * lane;

  float4 acc[kGatherCols];
#pragma unroll
  for (int cc = 0; cc < kGatherCols; ++cc) acc[cc] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (VEC && (tile + 1) * kGatherRows <= m)
    gather_cols<true>(acc, A, lda, m, n, b, cg, flat, colcnt, i0);
  else
    gather_cols<false>(acc, A, lda, m, n, b, cg, flat, colcnt, i0);

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = i0 + r;
    if (row >= m) break;
    const float zr = z ? zc * z[row] : 0.0f;
    float o[kGatherCols];
#pragma unroll
    for (int cc = 0; cc < kGatherCols; ++cc) {
      const float s = (r == 0) ? acc[cc].x : (r == 1) ? acc[cc].y : (r == 2) ? acc[cc].z : acc[cc].w;
      o[cc] = (cg * kGatherCols + cc < b) ? fmaf(scale, s, zr) : 0.0f;
    }
    *reinterpret_cast<float4 *>(out + row * (int64_t)kBld + cg * kGatherCols) =
        make_float4(o[0], o[1], o[2], o[3]);
  }
}

void launch_sketch_cols(const float *A, int64_t lda, int64_t m, int64_t n, int b,
                        const ChunkEntry *flat, const uint32_t *colcnt, float *out, float scale,
                        const float *z, float zc, hipStream_t st) {
  const int64_t tiles = (m + kGatherRows - 1) / kGatherRows;
  const int64_t nwaves = tiles * kGatherGroups;
  const int64_t nwg = (nwaves + 3) / 4;
  const bool vec = (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  if (vec)
    hipLaunchKernelGGL((sketch_cols_kernel<true>), dim3((unsigned)nwg), dim3(256), 0, st, A, lda, m,
                       n, b, flat, colcnt, out, nwaves, scale, z, zc);
  else
    hipLaunchKernelGGL((sketch_cols_kernel<false>), dim3((unsigned)nwg), dim3(256), 0, st, A, lda,
                       m, n, b, flat, colcnt, out, nwaves, scale, z, zc);
}

// ---------------------------------------------------------------- row sums
// rowsum[i] = sum_k A[i][k] in FP64: thread per row i of A (a column of the
// stored matrix, so a wave reads 256 contiguous bytes per stored row), K
// split over blockIdx.y; the splits are added in order by colsum_finish.
__global__ __launch_bounds__(256) void colsum_kernel(const float *__restrict__ A, int64_t lda,
                                                     int64_t m, int64_t n, int64_t rows_per_split,
                                                     double *__restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t split = blockIdx.y;
  if (i >= m) return;
  const int64_t k0 = split * rows_per_split;
  const int64_t k1 = (k0 + rows_per_split < n) ? k0 + rows_per_split : n;
  double s = 0.0;
  for (int64_t k = k0; k < k1; ++k) s += (double)A[k * lda + i];
  part[split * m + i] = s;
}

__global__ __launch_bounds__(256) void colsum_finish_kernel(const double *__restrict__ part,
                                                            int nsplit, int64_t m,
                                                            double *__restrict__ rowsum) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  double s = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) s += part[sp * m + i];
  rowsum[i] = s;
}

int colsum_num_splits(int64_t m, int64_t n) {
  const int64_t cb = (m + 255) / 256;
  int64_t ns = 1024 / cb;
  if (ns > 64) ns = 64;
  if (ns > n) ns = n;
  if (ns < 1) ns = 1;
  return (int)ns;
}

void launch_colsum(const float *A, int64_t lda, int64_t m, int64_t n, double *part, double *rowsum,
                   hipStream_t st) {
  const int ns0 = colsum_num_splits(m, n);
  const int64_t rps = (n + ns0 - 1) / ns0;
  const int ns = (int)((n + rps - 1) / rps);
  const unsigned cb = (unsigned)((m + 255) / 256);
  hipLaunchKernelGGL(colsum_kernel, dim3(cb, (unsigned)ns), dim3(256), 0, st, A, lda, m, n, rps,
                     part);
  hipLaunchKernelGGL(colsum_finish_kernel, dim3(cb), dim3(256), 0, st, part, ns, m, rowsum);
}

}  // namespace farpca_int
