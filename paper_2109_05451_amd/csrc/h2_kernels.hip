// HIP kernels of the H^2 matrix-vector product for CDNA4 (gfx950).
//
// Vector trees x^ and y^ (Section 3: one k-vector per node and vector) live
// in an H x nv column-major array; node c's entries are rows
// [hoff[c], hoff[c] + k).  The tree-ordered input copy and the dense-phase
// output are n x nv column-major.  Every output entry is produced by exactly
// one thread with a fixed summation order: no atomics, bitwise-reproducible
// results.
//
// Every phase of the product with op 'N' is one shape of work: a block row
// whose stored blocks are contiguous in HBM, i.e. one column-major
// nrows x ncols matrix M, times an input gathered block by block.  Leaf
// products (with the transposed leaf bases), the transfer up- and downsweep
// levels, the coupling products of all levels (Algorithm 4: levels are
// independent) and the dense leaf rows are all row lists of one streaming
// kernel; only the epilogue differs (store, accumulate, or the final
// permuted alpha/beta update).
#include <algorithm>
#include <type_traits>

#include "h2_internal.h"

namespace h2 {
namespace {

constexpr int kT = 256;  // threads per workgroup (4 wave64)

// X~[i, v] = X[perm[i], v]: the input in tree order (sub-vectors are taken
// from the node index sets, Section 3).
__global__ void k_permute_in(const double* __restrict__ X, int64_t ldx, const int32_t* __restrict__ perm,
                             double* __restrict__ xt, int64_t n, int64_t total) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t i = e % n, v = e / n;
  xt[e] = X[perm[i] + ldx * v];
}

__global__ void k_scale(double* __restrict__ Y, int64_t ldy, int64_t n, int64_t total, double beta) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t i = e % n, v = e / n;
  double* y = Y + i + ldy * v;
  *y = beta == 0.0 ? 0.0 : beta * *y;
}

// Vector loads of W consecutive elements (16 bytes for W = 16/sizeof(T)),
// nontemporal: the matrix data is streamed once per product.
template <typename T, int W> struct Vec { typedef T v __attribute__((ext_vector_type(W))); };
template <typename T> struct Vec<T, 1> { typedef T v; };
template <typename T, int W>
__device__ __forceinline__ typename Vec<T, W>::v ld_stream(const T* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const typename Vec<T, W>::v*>(p));
}
template <typename V>
__device__ __forceinline__ auto lane_elem(const V& v, int i) { return v[i]; }
__device__ __forceinline__ double lane_elem(const double& v, int) { return v; }
__device__ __forceinline__ float lane_elem(const float& v, int) { return v; }

// Accumulation type: FP64 data accumulates in FP64, FP32 data in FP32.
template <typename T> struct Acc { typedef T t; };

// Columns [0, cn) of M for one thread: rows W*p .. W*p+W-1 (one 16-byte
// load per column when W*sizeof(T) = 16), columns g, g+G, g+2G, ...  Four
// columns are loaded before any is used, so each thread keeps four loads in
// flight.
template <typename T, int NVB, int W, int XS>
__device__ __forceinline__ void stream_cols(const T* __restrict__ Mrow, int64_t m, int cn, int g, int G,
                                            const typename Acc<T>::t* xs, typename Acc<T>::t (&acc)[NVB][4]) {
  typedef typename Acc<T>::t A;
  typedef typename Vec<T, W>::v V;
  constexpr int U = 4;
  int j = g;
  for (; j + (U - 1) * G < cn; j += U * G) {
    V mv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) mv[u] = ld_stream<T, W>(Mrow + m * (j + u * G));
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int v = 0; v < NVB; ++v) {
        const A x = xs[v * XS + j + u * G];
#pragma unroll
        for (int r = 0; r < W; ++r) acc[v][r] = __builtin_fma((A)lane_elem(mv[u], r), x, acc[v][r]);
      }
  }
  for (; j < cn; j += G) {
    const V mv = ld_stream<T, W>(Mrow + m * j);
#pragma unroll
    for (int v = 0; v < NVB; ++v) {
      const A x = xs[v * XS + j];
#pragma unroll
      for (int r = 0; r < W; ++r) acc[v][r] = __builtin_fma((A)lane_elem(mv, r), x, acc[v][r]);
    }
  }
}

// The streaming kernel.  Workgroup = one row; thread (p, g) owns rows
// W*p .. W*p+W-1 of M and every G-th column.  The row's input is gathered
// into LDS chunk by chunk (block lookup by binary search over the row's
// block table, also in LDS); M is read once, with coalesced nontemporal
// 16-byte loads when the row's size and offset allow it.  Partial sums over
// g are combined in LDS in a fixed order, then the epilogue stores,
// accumulates, or applies the final permuted update
// Y[perm[i]] = alpha*(s + zn[i]) + beta*Y[perm[i]] (in FP64).
// T = double: the FP64 path; T = float: the low-rank phases of the FP32
// path (vector trees stay FP64 in memory; products accumulate in FP32).
// Rows are taken grid-stride: one workgroup per row, or fewer workgroups
// that each take several rows (a launch that holds only part of every CU).
template <typename T, int NVB>
__global__ __launch_bounds__(kT) void k_rows(const RowDesc* __restrict__ rows, int64_t nrows,
                                             const int32_t* __restrict__ colend,
                                             const int64_t* __restrict__ in_off, const T* __restrict__ data,
                                             const double* in, double* out, int nv, int mode, Epilogue ep) {
  typedef typename Acc<T>::t A;
  constexpr int VW = 16 / sizeof(T);                // elements per 16-byte load
  constexpr int XS = 2048 * 8 / sizeof(A) / NVB;    // LDS columns per chunk (16 KB)
  __shared__ A xs[XS * NVB];
  __shared__ int32_t s_end[kNbMax];
  __shared__ int64_t s_in[kNbMax];
  for (int64_t ri = blockIdx.x; ri < nrows; ri += gridDim.x) {
  __syncthreads();  // LDS of the previous row fully consumed
  const RowDesc R = rows[ri];
  const int m = R.nrows;
  if (m <= 0) continue;
  const int tid = threadIdx.x;
  const int nb = R.blk_end - R.blk_begin;  // <= kNbMax, checked when the schedule is built
  for (int i = tid; i < nb; i += kT) {
    s_end[i] = colend[R.blk_begin + i];
    s_in[i] = in_off[R.blk_begin + i];
  }
  __syncthreads();
  const int ncols = nb > 0 ? s_end[nb - 1] : 0;
  // widest row group that divides m and keeps the loads aligned
  int W = VW;
  while (W > 1 && ((m % W) != 0 || (R.data_off % W) != 0)) W >>= 1;
  const int P = m / W;
  const int G = kT / P;
  const int p = tid % P, g = tid / P;
  const T* Mrow = data + R.data_off + W * p;
  A acc[NVB][4];
#pragma unroll
  for (int v = 0; v < NVB; ++v)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[v][r] = 0;

  for (int c0 = 0; c0 < ncols; c0 += XS) {
    const int cn = min(XS, ncols - c0);
    if (c0 > 0) __syncthreads();  // previous chunk fully consumed
    for (int j = tid; j < cn; j += kT) {
      const int col = c0 + j;
      int lo = 0, hi = nb - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_end[mid] > col) hi = mid; else lo = mid + 1;
      }
      const int bstart = lo > 0 ? s_end[lo - 1] : 0;
      const double* src = in + s_in[lo] + (col - bstart);
#pragma unroll
      for (int v = 0; v < NVB; ++v) xs[v * XS + j] = v < nv ? (A)src[R.in_ld * v] : (A)0;
    }
    __syncthreads();
    if (g < G) {
      const T* Mc = Mrow + (int64_t)m * c0;
      if (W == VW) stream_cols<T, NVB, VW, XS>(Mc, m, cn, g, G, xs, acc);
      else if (VW >= 4 && W == 2) stream_cols<T, NVB, (VW >= 4 ? 2 : 1), XS>(Mc, m, cn, g, G, xs, acc);
      else stream_cols<T, NVB, 1, XS>(Mc, m, cn, g, G, xs, acc);
    }
  }
  __syncthreads();
  A* red = xs;  // G*m <= W*kT, so NVB*G*m <= XS*NVB
  if (g < G) {
#pragma unroll
    for (int v = 0; v < NVB; ++v)
      for (int r = 0; r < W; ++r) red[(v * G + g) * m + W * p + r] = acc[v][r];
  }
  __syncthreads();
  for (int o = tid; o < m * nv; o += kT) {
    const int a = o % m, v = o / m;
    A sa = 0;
    for (int gg = 0; gg < G; ++gg) sa += red[(v * G + gg) * m + a];
    double s = (double)sa;
    if (mode == MODE_STORE) {
      out[R.out_off + a + R.out_ld * v] = s;
    } else if (mode == MODE_ACCUM) {
      out[R.out_off + a + R.out_ld * v] += s;
    } else {
      const int64_t i = R.out_off + a;
      s += ep.zn[i + ep.n * v];
      double* y = ep.Y + ep.perm[i] + ep.ldy * v;
      *y = ep.beta == 0.0 ? ep.alpha * s : ep.alpha * s + ep.beta * *y;
    }
  }
  }  // rows
}

// Rows with more blocks than the LDS tables hold: one thread per output row
// and vector walks the columns (store mode only).
__global__ __launch_bounds__(kT) void k_rows_wide(const RowDesc* __restrict__ rows,
                                                  const int32_t* __restrict__ colend,
                                                  const int64_t* __restrict__ in_off,
                                                  const double* __restrict__ data, const double* in, double* out,
                                                  int nv) {
  const RowDesc R = rows[blockIdx.x];
  const int m = R.nrows;
  const int ncols = R.blk_end > R.blk_begin ? colend[R.blk_end - 1] : 0;
  for (int o = threadIdx.x; o < m * nv; o += kT) {
    const int a = o % m, v = o / m;
    double s = 0.0;
    int b = R.blk_begin, bstart = 0;
    for (int j = 0; j < ncols; ++j) {
      while (j >= colend[b]) bstart = colend[b++];
      s += data[R.data_off + a + (int64_t)m * j] * in[in_off[b] + (j - bstart) + R.in_ld * v];
    }
    out[R.out_off + a + R.out_ld * v] = s;
  }
}

// ---------------------------------------------------------------------------
// Multi-vector path (FP64 MFMA).  Vector trees and the tree-ordered input and
// dense partial are row-major with NVP = 16*NT vectors per row (padding
// vectors are zero).  The same row lists as the streaming kernel are used:
// out (m x NVP) = M (m x ncols, column-major) * B (ncols x NVP, gathered).
// 16x16x4 MFMA lane layouts (wave64, measured on gfx950): A[i][k] at lane
// i + 16k, B[k][j] at lane j + 16k; accumulator element r (0..3) of lane l
// holds C[4r + l/16][l%16] for v_mfma_f64_16x16x4f64 and
// C[4(l/16) + r][l%16] for v_mfma_f32_16x16x4f32.
typedef double d4 __attribute__((ext_vector_type(4)));

// X~ (tree order, row-major NVP) from X (original order, column-major):
// thread per original index j reads X[j, v] (coalesced over j) and writes
// the row of tree position pinv[j].
// Permutations of the multi-vector path through an LDS tile of 64 points x
// nvp vectors, so that both the column-major side (64 consecutive points of
// one vector) and the tree-ordered side (one point's nvp vectors, contiguous)
// are accessed with coalesced loads and stores.

// xt[pinv[j], v] = X[j, v] for v < nv, 0 for nv <= v < NVP.  A workgroup
// moves kPermTile original rows through LDS: every thread issues all of its
// coalesced column loads first (PER of them, unrolled), then the wave-wide
// row stores follow.
template <int NVP>
__global__ __launch_bounds__(256) void k_permute_in_rm(const double* __restrict__ X, int64_t ldx,
                                                       const int32_t* __restrict__ pinv, double* __restrict__ xt,
                                                       int64_t n, int nv) {
  constexpr int LD = NVP + 1, PER = kPermTile * NVP / 256;
  __shared__ double tile[kPermTile * LD];
  const int64_t j0 = blockIdx.x * (int64_t)kPermTile;
  const int rows = (int)min<int64_t>(kPermTile, n - j0);
  double r[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, v = e / kPermTile, jj = e - v * kPermTile;
    r[i] = jj < rows && v < nv ? __builtin_nontemporal_load(X + j0 + jj + ldx * v) : 0.0;
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, v = e / kPermTile, jj = e - v * kPermTile;
    tile[jj * LD + v] = r[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, jj = e / NVP, v = e - jj * NVP;
    if (jj < rows) xt[(int64_t)pinv[j0 + jj] * NVP + v] = tile[jj * LD + v];
  }
}

// Y[j, v] = alpha * Z[pinv[j], v] + beta * Y[j, v] (Z row-major NVP, tree
// order), the same way round: row gathers into LDS, column stores out.
template <int NVP>
__global__ __launch_bounds__(256) void k_permute_out_rm(const double* __restrict__ Z,
                                                        const int32_t* __restrict__ pinv, double alpha, double beta,
                                                        double* __restrict__ Y, int64_t ldy, int64_t n, int nv) {
  constexpr int LD = NVP + 1, PER = kPermTile * NVP / 256;
  __shared__ double tile[kPermTile * LD];
  const int64_t j0 = blockIdx.x * (int64_t)kPermTile;
  const int rows = (int)min<int64_t>(kPermTile, n - j0);
  double r[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, jj = e / NVP, v = e - jj * NVP;
    r[i] = jj < rows && v < nv ? __builtin_nontemporal_load(Z + (int64_t)pinv[j0 + jj] * NVP + v) : 0.0;
  }
  double yv[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, v = e / kPermTile, jj = e - v * kPermTile;
    yv[i] = beta != 0.0 && jj < rows && v < nv ? Y[j0 + jj + ldy * v] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, jj = e / NVP, v = e - jj * NVP;
    tile[jj * LD + v] = r[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, v = e / kPermTile, jj = e - v * kPermTile;
    if (jj < rows && v < nv) {
      const double z = alpha * tile[jj * LD + v];
      Y[j0 + jj + ldy * v] = beta == 0.0 ? z : z + beta * yv[i];
    }
  }
}

typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<double> { typedef d4 t; };
template <> struct MfmaAcc<float> { typedef f4 t; };
__device__ __forceinline__ d4 mfma16x16x4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16x16x4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Four 4x4x4 FP64 products in one instruction.  Lane 16k + 4*blk + i holds
// A_blk[i][k], lane 16k + 4*blk + j holds B_blk[k][j], and the result of
// lane 16i + 4*blk + j is D_blk[i][j].
__device__ __forceinline__ double mfma4x4x4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// T = double: FP64 MFMA; T = float: FP32 MFMA on the FP32 copy of the
// low-rank data (inputs rounded to FP32 when staged, FP32 accumulation).
// Rows are taken grid-stride (row = blockIdx.x, blockIdx.x + gridDim.x, ...):
// with one workgroup per row this is a plain launch, with fewer workgroups
// it is a persistent kernel.  KC is the number of columns staged per LDS
// chunk (KC/4 MFMA k-steps).
template <typename T, int NT, int MAXT, int KC>
__global__ __launch_bounds__(kT) void k_rows_mfma(const RowDesc* __restrict__ rows, int64_t nrows,
                                                  const int32_t* __restrict__ colend,
                                                  const int64_t* __restrict__ in_off,
                                                  const T* __restrict__ data, const double* in, double* out,
                                                  int mode, int remap) {
  typedef typename MfmaAcc<T>::t CT;
  constexpr int NVP = 16 * NT;
  __shared__ T bs[KC * NVP];
  __shared__ int32_t s_end[kNbMax];
  __shared__ int64_t s_in[kNbMax];
  __shared__ int64_t s_src[KC];  // input row of each column of the chunk
  // rows by workgroup: plain grid-stride, or (remap) each XCD (workgroups
  // b with the same b % 8) takes one contiguous eighth of the rows, so that
  // neighbouring rows, which share input segments, meet in the same L2
  const int64_t per = remap ? (nrows + 7) / 8 : nrows;
  const int64_t xcd = remap ? blockIdx.x % 8 : 0;
  const int64_t step = remap ? gridDim.x / 8 : gridDim.x;
  for (int64_t jr = remap ? blockIdx.x / 8 : blockIdx.x; jr < per; jr += step) {
    const int64_t ri = xcd * per + jr;
    if (ri >= nrows) break;
  __syncthreads();  // LDS of the previous row fully consumed
  const RowDesc R = rows[ri];
  const int m = R.nrows;
  if (m <= 0) continue;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = R.blk_end - R.blk_begin;
  for (int i = tid; i < nb; i += kT) {
    s_end[i] = colend[R.blk_begin + i];
    s_in[i] = in_off[R.blk_begin + i];
  }
  __syncthreads();
  const int ncols = nb > 0 ? s_end[nb - 1] : 0;
  const int mt = (m + 15) >> 4;  // 16-row tiles of M; waves take tiles w, w+4, ... (at most MAXT each)
  CT acc[MAXT][NT];
#pragma unroll
  for (int i = 0; i < MAXT; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = CT{0, 0, 0, 0};
  const int arow = lane & 15, akk = lane >> 4;  // A fragment: row within tile, k within step
  const T* M = data + R.data_off;

  for (int c0 = 0; c0 < ncols; c0 += KC) {
    const int cn = min(KC, ncols - c0);
    if (c0 > 0) __syncthreads();
    if (tid < cn) {
      const int col = c0 + tid;
      int lo = 0, hi = nb - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_end[mid] > col) hi = mid; else lo = mid + 1;
      }
      s_src[tid] = s_in[lo] + (col - (lo > 0 ? s_end[lo - 1] : 0));
    }
    __syncthreads();
    for (int e = tid; e < KC * NVP; e += kT) {
      const int j = e / NVP, v = e - j * NVP;
      bs[e] = j < cn ? (T)in[s_src[j] * NVP + v] : (T)0;
    }
    __syncthreads();
    const int nsteps = (cn + 3) >> 2;
#pragma unroll
    for (int ti = 0; ti < MAXT; ++ti) {
      const int tile = wave + 4 * ti;
      if (tile >= mt) break;
      const int r = tile * 16 + arow;
      const bool rok = r < m;
      const T* Ar = M + r + (int64_t)m * c0;
      int s = 0;
      for (; s + 3 < nsteps; s += 4) {
        T a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int col = 4 * (s + u) + akk;
          a[u] = (rok && col < cn) ? __builtin_nontemporal_load(Ar + (int64_t)m * col) : (T)0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            const T b = bs[(4 * (s + u) + akk) * NVP + 16 * j + arow];
            acc[ti][j] = mfma16x16x4(a[u], b, acc[ti][j]);
          }
      }
      for (; s < nsteps; ++s) {
        const int col = 4 * s + akk;
        const T a = (rok && col < cn) ? __builtin_nontemporal_load(Ar + (int64_t)m * col) : (T)0;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
          const T b = bs[(4 * s + akk) * NVP + 16 * j + arow];
          acc[ti][j] = mfma16x16x4(a, b, acc[ti][j]);
        }
      }
    }
  }
  // epilogue: accumulator element r of the lane is row 4r + lane/16 (FP64)
  // or 4*(lane/16) + r (FP32) of each of its tiles, column lane%16
#pragma unroll
  for (int ti = 0; ti < MAXT; ++ti) {
    const int tile = wave + 4 * ti;
    if (tile >= mt) break;
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = tile * 16 + (sizeof(T) == 8 ? 4 * r + akk : 4 * akk + r);
        if (a < m) {
          double* o = out + (R.out_off + a) * NVP + 16 * j + arow;
          if (mode == MODE_STORE) *o = (double)acc[ti][j][r];
          else *o += (double)acc[ti][j][r];
        }
      }
  }
  }  // rows
}

// Software-pipelined variant for 64 vectors: the input chunk (32 columns x
// 64 vectors) is double-buffered in LDS; the next chunk's gather is issued
// into registers before the current chunk's MFMAs and stored after them, so
// one barrier per chunk separates the buffers.  Wave w gathers columns
// w, w + 4, ... of a chunk, one column (64 contiguous vectors) per load
// instruction, and finds each column's block with a cursor that only moves
// forward (columns increase), instead of a search per chunk.
template <typename T, int MAXT>
__global__ __launch_bounds__(kT) void k_rows_mfma_pipe(const RowDesc* __restrict__ rows, int64_t nrows,
                                                       const int32_t* __restrict__ colend,
                                                       const int64_t* __restrict__ in_off,
                                                       const T* __restrict__ data, const double* in, double* out,
                                                       int mode, int remap) {
  typedef typename MfmaAcc<T>::t CT;
  constexpr int NT = 4, NVP = 64, KC = 32, PER = KC / 4;  // PER columns per wave per chunk
  __shared__ T bs[2][KC * NVP];
  __shared__ int32_t s_end[kNbMax];
  __shared__ int64_t s_in[kNbMax];
  const int64_t per = remap ? (nrows + 7) / 8 : nrows;
  const int64_t xcd = remap ? blockIdx.x % 8 : 0;
  const int64_t step = remap ? gridDim.x / 8 : gridDim.x;
  for (int64_t jr = remap ? blockIdx.x / 8 : blockIdx.x; jr < per; jr += step) {
    const int64_t ri = xcd * per + jr;
    if (ri >= nrows) break;
    __syncthreads();  // LDS of the previous row fully consumed
    const RowDesc R = rows[ri];
    const int m = R.nrows;
    if (m <= 0) continue;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = R.blk_end - R.blk_begin;
    for (int i = tid; i < nb; i += kT) {
      s_end[i] = colend[R.blk_begin + i];
      s_in[i] = in_off[R.blk_begin + i];
    }
    __syncthreads();
    const int ncols = nb > 0 ? s_end[nb - 1] : 0;
    const int nch = (ncols + KC - 1) / KC;
    const int mt = (m + 15) >> 4;
    CT acc[MAXT][NT];
#pragma unroll
    for (int i = 0; i < MAXT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = CT{0, 0, 0, 0};
    const int arow = lane & 15, akk = lane >> 4;
    const T* M = data + R.data_off;
    int bw = 0;  // this wave's block cursor
    T reg[PER];
    auto gather = [&](int c) {
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int col = c * KC + wave + 4 * i;
        T v = (T)0;
        if (col < ncols) {
          while (s_end[bw] <= col) ++bw;
          const int64_t src = s_in[bw] + (col - (bw > 0 ? s_end[bw - 1] : 0));
          v = (T)in[src * NVP + lane];
        }
        reg[i] = v;
      }
    };
    auto store = [&](int buf) {
#pragma unroll
      for (int i = 0; i < PER; ++i) bs[buf][(wave + 4 * i) * NVP + lane] = reg[i];
    };
    if (nch > 0) {
      gather(0);
      store(0);
    }
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
      const int buf = c & 1;
      const int c0 = c * KC, cn = min(KC, ncols - c0);
      if (c + 1 < nch) gather(c + 1);
      const int nsteps = (cn + 3) >> 2;
#pragma unroll
      for (int ti = 0; ti < MAXT; ++ti) {
        const int tile = wave + 4 * ti;
        if (tile >= mt) break;
        const int r = tile * 16 + arow;
        const bool rok = r < m;
        const T* Ar = M + r + (int64_t)m * c0;
        T a[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int col = 4 * u + akk;
          a[u] = (rok && col < cn) ? __builtin_nontemporal_load(Ar + (int64_t)m * col) : (T)0;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          if (u < nsteps) {
#pragma unroll
            for (int j = 0; j < NT; ++j) {
              const T b = bs[buf][(4 * u + akk) * NVP + 16 * j + arow];
              acc[ti][j] = mfma16x16x4(a[u], b, acc[ti][j]);
            }
          }
        }
      }
      if (c + 1 < nch) store(buf ^ 1);
      __syncthreads();
    }
#pragma unroll
    for (int ti = 0; ti < MAXT; ++ti) {
      const int tile = wave + 4 * ti;
      if (tile >= mt) break;
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = tile * 16 + (sizeof(T) == 8 ? 4 * r + akk : 4 * akk + r);
          if (a < m) {
            double* o = out + (R.out_off + a) * NVP + 16 * j + arow;
            if (mode == MODE_STORE) *o = (double)acc[ti][j][r];
            else *o += (double)acc[ti][j][r];
          }
        }
    }
  }
}

// Balanced variant for 64 vectors and rows of at most 64 outputs: wave w
// owns vector tile w (16 vectors) for every 16-row tile of the row, so all
// four waves issue MFMAs whatever the row count (a 36-row block gives each
// wave three tiles instead of leaving one wave idle).  Both operands of a
// chunk of KC columns go through LDS, double-buffered: the matrix chunk is a
// contiguous m x KC slice (coalesced loads), the gathered input chunk is
// KC x 64; the next chunk is loaded into registers before the current
// chunk's MFMAs and stored after them, with one barrier per chunk.  OCC > 1
// asks the compiler for registers enough for OCC workgroups per CU (four fit
// the 16-column chunk's LDS, more the 8-column one's), trading a little
// spilling for latency hiding.  The gathered input is read as TI: FP64, or
// FP32 in the FP32 variant's coupling launches.  With FP32 data each
// gathered value is rounded to FP32 anyway, so gathering from a rounded copy
// of x^ gives the same products from half the bytes.
template <typename T, typename TI, int KC, bool DEEP, int MT, int OCC>
__global__ __launch_bounds__(kT, OCC) void k_rows_mfma_bal(const RowDesc* __restrict__ rows, int64_t nrows,
                                                      const int32_t* __restrict__ colend,
                                                      const int64_t* __restrict__ in_off,
                                                      const T* __restrict__ data, const TI* in, double* out,
                                                      int mode, int remap) {
  typedef typename MfmaAcc<T>::t CT;
  constexpr int NVP = 64, LDA = 68, LDB = 66;  // padded LDS rows (doubles or floats)
  constexpr int PA = (64 * KC + kT - 1) / kT;   // matrix elements per thread per chunk (m <= 64)
  constexpr int PB = KC / 4;                     // gathered columns per wave per chunk
  __shared__ T sa[2][KC * LDA];
  __shared__ T sb[2][KC * LDB];
  __shared__ int32_t s_end[kNbMax];
  __shared__ int64_t s_in[kNbMax];
  const int64_t per = remap ? (nrows + 7) / 8 : nrows;
  const int64_t xcd = remap ? blockIdx.x % 8 : 0;
  const int64_t step = remap ? gridDim.x / 8 : gridDim.x;
  for (int64_t jr = remap ? blockIdx.x / 8 : blockIdx.x; jr < per; jr += step) {
    const int64_t ri = xcd * per + jr;
    if (ri >= nrows) break;
    __syncthreads();
    const RowDesc R = rows[ri];
    const int m = R.nrows;
    if (m <= 0) continue;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = R.blk_end - R.blk_begin;
    for (int i = tid; i < nb; i += kT) {
      s_end[i] = colend[R.blk_begin + i];
      s_in[i] = in_off[R.blk_begin + i];
    }
    __syncthreads();
    const int ncols = nb > 0 ? s_end[nb - 1] : 0;
    const int nch = (ncols + KC - 1) / KC;
    const int mt = (m + 15) >> 4;
    CT acc[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) acc[i] = CT{0, 0, 0, 0};
    // FP64 rows of 33-36 outputs (rank 36): rows 32-35 go through the 4x4x4
    // instruction (its four blocks are four 4-vector groups sharing the same
    // A rows) instead of a 16-row tile that is three quarters padding.  Not
    // in the one-workgroup-per-CU forms: compiled there, the extra
    // accumulator lands in an AGPR that the epilogue read before the MFMA's
    // result wait states.
    constexpr bool kTail4 = sizeof(T) == 8 && MT == 3 && OCC > 1;
    const bool tail4 = kTail4 && m > 32 && m <= 36;
    double acc4 = 0.0;
    const int arow = lane & 15, akk = lane >> 4;
    const T* M = data + R.data_off;
    int bw = 0;
    T ra[PA], rb[PB];
    auto load = [&](int c, T* ra, T* rb) {
      const int c0 = c * KC, cn = min(KC, ncols - c0);
      const int64_t base = (int64_t)m * c0;  // the chunk is m * cn contiguous elements
#pragma unroll
      for (int i = 0; i < PA; ++i) {
        const int e = tid + kT * i;
        ra[i] = e < m * cn ? __builtin_nontemporal_load(M + base + e) : (T)0;
      }
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const int col = c0 + wave + 4 * i;
        T v = (T)0;
        if (col < ncols) {
          while (s_end[bw] <= col) ++bw;
          const int64_t src = s_in[bw] + (col - (bw > 0 ? s_end[bw - 1] : 0));
          v = (T)in[src * NVP + lane];
        }
        rb[i] = v;
      }
    };
    auto store = [&](int buf, int c, const T* ra, const T* rb) {
      const int cn = min(KC, ncols - c * KC);
#pragma unroll
      for (int i = 0; i < PA; ++i) {
        const int e = tid + kT * i;
        if (e < m * KC) {
          const int col = e / m, row = e - col * m;
          sa[buf][col * LDA + row] = col < cn ? ra[i] : (T)0;
        }
      }
#pragma unroll
      for (int i = 0; i < PB; ++i) sb[buf][(wave + 4 * i) * LDB + lane] = rb[i];
    };
    // rows m .. 16*mt of the A tiles read zeros
    for (int e = tid; e < 2 * KC * LDA; e += kT) {
      const int row = e % LDA;
      if (row >= m) (&sa[0][0])[e] = (T)0;
    }
    auto compute = [&](int c) {
      const int buf = c & 1;
      const int cn = min(KC, ncols - c * KC);
      const int nsteps = (cn + 3) >> 2;
      const T* A = sa[buf];
      const T* B = sb[buf];
#pragma unroll
      for (int u = 0; u < KC / 4; ++u) {
        if (u < nsteps) {
          const int k = 4 * u + akk;
          const T b = B[k * LDB + 16 * wave + arow];
#pragma unroll
          for (int ti = 0; ti < MT; ++ti) {
            if (ti >= mt) continue;
            if constexpr (kTail4) {
              if (ti == 2 && tail4) {
                acc4 = mfma4x4x4(A[k * LDA + 32 + (arow & 3)], b, acc4);
                continue;
              }
            }
            acc[ti] = mfma16x16x4(A[k * LDA + 16 * ti + arow], b, acc[ti]);
          }
        }
      }
    };
    if (!DEEP) {
      if (nch > 0) {
        load(0, ra, rb);
        store(0, 0, ra, rb);
      }
      __syncthreads();
      for (int c = 0; c < nch; ++c) {
        if (c + 1 < nch) load(c + 1, ra, rb);
        compute(c);
        if (c + 1 < nch) store((c + 1) & 1, c + 1, ra, rb);
        __syncthreads();
      }
    } else {
      // two register sets: chunk c+2 is loaded while chunk c is multiplied
      // and chunk c+1 (loaded an iteration earlier) is stored
      T ra2[PA], rb2[PB];
      if (nch > 0) {
        load(0, ra, rb);
        store(0, 0, ra, rb);
      }
      if (nch > 1) load(1, ra2, rb2);
      __syncthreads();
      for (int c = 0; c < nch; c += 2) {
        if (c + 2 < nch) load(c + 2, ra, rb);
        compute(c);
        if (c + 1 < nch) store(1, c + 1, ra2, rb2);
        __syncthreads();
        if (c + 1 >= nch) break;
        if (c + 3 < nch) load(c + 3, ra2, rb2);
        compute(c + 1);
        if (c + 2 < nch) store(0, c + 2, ra, rb);
        __syncthreads();
      }
    }
#pragma unroll
    for (int ti = 0; ti < MT; ++ti) {
      if (ti >= mt) break;
      if (ti == 2 && tail4) {
        const int a = 32 + akk;  // row of this lane's 4x4x4 result
        if (a < m) {
          double* o = out + (R.out_off + a) * NVP + 16 * wave + arow;
          if (mode == MODE_STORE) *o = acc4;
          else *o += acc4;
        }
        continue;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = ti * 16 + (sizeof(T) == 8 ? 4 * r + akk : 4 * akk + r);
        if (a < m) {
          double* o = out + (R.out_off + a) * NVP + 16 * wave + arow;
          if (mode == MODE_STORE) *o = (double)acc[ti][r];
          else *o += (double)acc[ti][r];
        }
      }
    }
  }
}

// Transposed block-column product (op 'T') for the coupling and dense
// phases: out[b, v] = sum over the blocks of the column, sum_a Mblk[a, b]
// x_blk[a, v].  Each stored block (mr x ms, column-major, contiguous) is
// copied into LDS with coalesced loads, its input segment too, then thread
// (b, q) sums rows a = q, q+Q, ... of column b; column b sits at LDS offset
// b*(mr+1) so that neighbouring lanes hit different banks.  Partials over q
// are combined in a fixed order: deterministic, no atomics.
template <typename T, int NVB>
__global__ __launch_bounds__(kT) void k_rows_t(const RowDesc* __restrict__ rows, const int64_t* __restrict__ bdata,
                                               const int32_t* __restrict__ bmr, const int64_t* __restrict__ bin,
                                               const T* __restrict__ data, const double* in, double* out,
                                               int nv) {
  typedef typename Acc<T>::t A;
  constexpr int LDSD = 4352;  // elements: a 64 x 64 block with padding (64*65 = 4160) and slack
  __shared__ A blk[LDSD];
  __shared__ A xs[NVB * kMaxDim];
  const RowDesc R = rows[blockIdx.x];
  const int ms = R.nrows;
  if (ms <= 0) return;
  const int tid = threadIdx.x;
  const int Q = kT / ms;
  const int b = tid % ms, q = tid / ms;
  A acc[NVB];
#pragma unroll
  for (int v = 0; v < NVB; ++v) acc[v] = 0;
  for (int k = R.blk_begin; k < R.blk_end; ++k) {
    const int mr = bmr[k];
    const T* M = data + bdata[k];
    const double* x = in + bin[k];
    // rows handled per LDS pass, so that (rows+1)*ms fits
    const int rows_per = min(mr, LDSD / ms - 1);
    for (int a0 = 0; a0 < mr; a0 += rows_per) {
      const int ra = min(rows_per, mr - a0);
      __syncthreads();  // previous pass consumed
      for (int e = tid; e < ra * ms; e += kT) {
        const int cb = e / ra, ca = e - cb * ra;
        blk[cb * (ra + 1) + ca] = __builtin_nontemporal_load(M + a0 + ca + (int64_t)mr * cb);
      }
      for (int e = tid; e < ra * NVB; e += kT) {
        const int v = e / ra, a = e - v * ra;
        xs[v * kMaxDim + a] = v < nv ? (A)x[a0 + a + R.in_ld * v] : (A)0;
      }
      __syncthreads();
      if (q < Q) {
        const A* col = blk + b * (ra + 1);
        for (int a = q; a < ra; a += Q) {
          const A mv = col[a];
#pragma unroll
          for (int v = 0; v < NVB; ++v) acc[v] = __builtin_fma(mv, xs[v * kMaxDim + a], acc[v]);
        }
      }
    }
  }
  __syncthreads();
  A* red = blk;  // Q*ms <= kT, so NVB*Q*ms <= LDSD for NVB <= 16
  if (q < Q) {
#pragma unroll
    for (int v = 0; v < NVB; ++v) red[(v * Q + q) * ms + b] = acc[v];
  }
  __syncthreads();
  for (int o = tid; o < ms * nv; o += kT) {
    const int bb = o % ms, v = o / ms;
    A s = 0;
    for (int qq = 0; qq < Q; ++qq) s += red[(v * Q + qq) * ms + bb];
    out[R.out_off + bb + R.out_ld * v] = (double)s;
  }
}

inline unsigned grid1d(int64_t total, int threads) { return (unsigned)((total + threads - 1) / threads); }

// Workgroups of a row launch: `grid` (0 = one per row) capped at the rows;
// with the XCD remap a multiple of 8 covering eight equal row ranges.
inline int64_t grid_of_rows(int64_t nrows, int64_t grid, int remap) {
  int64_t g = grid > 0 && grid < nrows ? grid : nrows;
  if (remap) {
    const int64_t per = (nrows + 7) / 8;
    g = std::min<int64_t>((g + 7) / 8 * 8, 8 * per);
  }
  return g;
}

}  // namespace

hipError_t launch_permute_in(const double* X, int64_t ldx, const int32_t* perm, double* xt, int64_t n, int nv,
                             hipStream_t s) {
  const int64_t total = n * nv;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute_in, dim3(grid1d(total, 256)), dim3(256), 0, s, X, ldx, perm, xt, n, total);
  return hipGetLastError();
}

hipError_t launch_scale(double* Y, int64_t ldy, int64_t n, int64_t nv, double beta, hipStream_t s) {
  const int64_t total = n * nv;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale, dim3(grid1d(total, 256)), dim3(256), 0, s, Y, ldy, n, total, beta);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rows(const RowDesc* rows, int64_t nrows, const int32_t* colend, const int64_t* in_off,
                       const T* data, const double* in, double* out, int nv, int mode, const Epilogue& ep,
                       hipStream_t s, int64_t grid) {
  if (nrows == 0) return hipSuccess;
  const dim3 g((unsigned)(grid > 0 && grid < nrows ? grid : nrows)), block(kT);
  if (nv <= 1)
    hipLaunchKernelGGL((k_rows<T, 1>), g, block, 0, s, rows, nrows, colend, in_off, data, in, out, nv, mode, ep);
  else if (nv == 2)
    hipLaunchKernelGGL((k_rows<T, 2>), g, block, 0, s, rows, nrows, colend, in_off, data, in, out, nv, mode, ep);
  else if (nv <= 4)
    hipLaunchKernelGGL((k_rows<T, 4>), g, block, 0, s, rows, nrows, colend, in_off, data, in, out, nv, mode, ep);
  else
    return hipErrorInvalidValue;  // callers pass at most kPassVectors vectors
  return hipGetLastError();
}
template hipError_t launch_rows<double>(const RowDesc*, int64_t, const int32_t*, const int64_t*, const double*,
                                        const double*, double*, int, int, const Epilogue&, hipStream_t, int64_t);
template hipError_t launch_rows<float>(const RowDesc*, int64_t, const int32_t*, const int64_t*, const float*,
                                       const double*, double*, int, int, const Epilogue&, hipStream_t, int64_t);

template <typename T>
hipError_t launch_rows_mfma(const RowDesc* rows, int64_t nrows, const int32_t* colend, const int64_t* in_off,
                            const T* data, const double* in, double* out, int nvp, int mode, int max_rows,
                            hipStream_t s, int kc, int64_t grid, int remap, const float* in32) {
  if (nrows == 0) return hipSuccess;
  const dim3 g((unsigned)grid_of_rows(nrows, grid, remap)), block(kT);
#define H2_MFMA3(NT, MAXT, KC)                                                                                   \
  hipLaunchKernelGGL((k_rows_mfma<T, NT, MAXT, KC>), g, block, 0, s, rows, nrows, colend, in_off, data, in, out, \
                     mode, remap)
#define H2_MFMA(NT)                                     \
  do {                                                  \
    if (max_rows <= 64) {                               \
      if (kc == 32) H2_MFMA3(NT, 1, 32);                \
      else H2_MFMA3(NT, 1, 64);                         \
    } else {                                            \
      if (kc == 32) H2_MFMA3(NT, 4, 32);                \
      else H2_MFMA3(NT, 4, 64);                         \
    }                                                   \
  } while (0)
  // kc: 32 or 64 columns per chunk; 0: pipelined kernel; 1, 2: balanced
  // kernel with 32 or 16 columns; 3, 4: balanced, 16 or 32 columns, loads
  // issued two chunks ahead; 5, 6: balanced, 16 columns (loads one or two
  // chunks ahead) with registers for four workgroups per CU; 7, 8: the same
  // with 8 columns and five workgroups per CU (0-8 take 64 vectors, 1-8 rows
  // of at most 64 outputs; other launches fall back to 64 columns).  in32:
  // an FP32 copy of the input that the balanced kernels read instead (FP32
  // data only; null: read in)
  if ((kc == 0 && nvp != 64) || ((kc >= 1 && kc <= 8) && (nvp != 64 || max_rows > 64))) kc = 64;
  if (kc >= 1 && kc <= 8) {
#define H2_BAL(KCV, DEEP, MT, OCC)                                                                           \
  do {                                                                                                       \
    if constexpr (std::is_same<T, float>::value) {                                                           \
      if (in32) {                                                                                            \
        hipLaunchKernelGGL((k_rows_mfma_bal<T, float, KCV, DEEP, MT, OCC>), g, block, 0, s, rows, nrows, colend, \
                           in_off, data, in32, out, mode, remap);                                           \
        break;                                                                                               \
      }                                                                                                      \
    }                                                                                                        \
    hipLaunchKernelGGL((k_rows_mfma_bal<T, double, KCV, DEEP, MT, OCC>), g, block, 0, s, rows, nrows, colend,  \
                       in_off, data, in, out, mode, remap);                                                 \
  } while (0)
#define H2_BAL_MT(KCV, DEEP, OCC)                       \
  do {                                                  \
    if (max_rows <= 16) H2_BAL(KCV, DEEP, 1, OCC);      \
    else if (max_rows <= 32) H2_BAL(KCV, DEEP, 2, OCC); \
    else if (max_rows <= 48) H2_BAL(KCV, DEEP, 3, OCC); \
    else H2_BAL(KCV, DEEP, 4, OCC);                     \
  } while (0)
    if (kc == 1) H2_BAL_MT(32, false, 1);
    else if (kc == 2) H2_BAL_MT(16, false, 1);
    else if (kc == 3) H2_BAL_MT(16, true, 1);
    else if (kc == 4) H2_BAL_MT(32, true, 1);
    else if (kc == 5) H2_BAL_MT(16, false, 4);
    else if (kc == 6) H2_BAL_MT(16, true, 4);
    else if (kc == 7) H2_BAL_MT(8, false, 5);
    else H2_BAL_MT(8, true, 5);
#undef H2_BAL_MT
#undef H2_BAL
    return hipGetLastError();
  }
  if (kc == 0) {
    if (max_rows <= 64)
      hipLaunchKernelGGL((k_rows_mfma_pipe<T, 1>), g, block, 0, s, rows, nrows, colend, in_off, data, in, out, mode,
                         remap);
    else
      hipLaunchKernelGGL((k_rows_mfma_pipe<T, 4>), g, block, 0, s, rows, nrows, colend, in_off, data, in, out, mode,
                         remap);
    return hipGetLastError();
  }
  switch (nvp) {
    case 16: H2_MFMA(1); break;
    case 32: H2_MFMA(2); break;
    case 48: H2_MFMA(3); break;
    case 64: H2_MFMA(4); break;
    default: return hipErrorInvalidValue;
  }
#undef H2_MFMA
#undef H2_MFMA3
  return hipGetLastError();
}
template hipError_t launch_rows_mfma<double>(const RowDesc*, int64_t, const int32_t*, const int64_t*, const double*,
                                             const double*, double*, int, int, int, hipStream_t, int, int64_t, int,
                                             const float*);
template hipError_t launch_rows_mfma<float>(const RowDesc*, int64_t, const int32_t*, const int64_t*, const float*,
                                            const double*, double*, int, int, int, hipStream_t, int, int64_t, int,
                                            const float*);


// Batched permutations through an LDS tile of kPermTile original rows of one
// operator: workgroup b takes tile b of the list (operator tile_op[b], first
// original row tile_j0[b]), so no workgroup idles on a small operator, and
// both the column-major side (64 consecutive points of one vector) and the
// row-major workspace side (one point's NVP vectors) are accessed with
// coalesced loads and stores.  In: rows xt_row + pinv[j] get X[j, v] for
// v < nv, zeros for the padding vectors (and for nv == 0 or alpha == 0, when
// X is not read).  Out: Y[j, v] = alpha Z[zn_row + pinv[j], v] + beta Y[j, v]
// for v < nv (beta == 0: Y not read).
template <int NVP>
__global__ __launch_bounds__(256) void k_batch_permute_in(const BatchItem* __restrict__ items,
                                                          const int32_t* __restrict__ tile_op,
                                                          const int32_t* __restrict__ tile_j0,
                                                          const int32_t* __restrict__ pinv, double* __restrict__ ws) {
  constexpr int LD = NVP + 1, PER = kPermTile * NVP / 256;
  __shared__ double tile[kPermTile * LD];
  const BatchItem it = items[tile_op[blockIdx.x]];
  const int64_t j0 = tile_j0[blockIdx.x];
  const int rows = (int)min<int64_t>(kPermTile, it.n - j0);
  const int nv = (it.nv > 0 && it.alpha != 0.0) ? (int)it.nv : 0;
  double r[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, v = e / kPermTile, jj = e - v * kPermTile;
    r[i] = jj < rows && v < nv ? __builtin_nontemporal_load(it.X + j0 + jj + it.ldx * v) : 0.0;
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, v = e / kPermTile, jj = e - v * kPermTile;
    tile[jj * LD + v] = r[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, jj = e / NVP, v = e - jj * NVP;
    if (jj < rows) ws[(it.xt_row + pinv[it.pinv_off + j0 + jj]) * NVP + v] = tile[jj * LD + v];
  }
}

template <int NVP>
__global__ __launch_bounds__(256) void k_batch_permute_out(const BatchItem* __restrict__ items,
                                                           const int32_t* __restrict__ tile_op,
                                                           const int32_t* __restrict__ tile_j0,
                                                           const int32_t* __restrict__ pinv,
                                                           const double* __restrict__ ws) {
  constexpr int LD = NVP + 1, PER = kPermTile * NVP / 256;
  __shared__ double tile[kPermTile * LD];
  const BatchItem it = items[tile_op[blockIdx.x]];
  if (it.nv <= 0) return;  // the operator is skipped: Y untouched (uniform over the workgroup)
  const int64_t j0 = tile_j0[blockIdx.x];
  const int rows = (int)min<int64_t>(kPermTile, it.n - j0);
  const int nv = (int)it.nv;
  double r[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, jj = e / NVP, v = e - jj * NVP;
    r[i] = jj < rows && v < nv && it.alpha != 0.0
               ? __builtin_nontemporal_load(ws + (it.zn_row + pinv[it.pinv_off + j0 + jj]) * NVP + v)
               : 0.0;
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, jj = e / NVP, v = e - jj * NVP;
    tile[jj * LD + v] = r[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = threadIdx.x + 256 * i, v = e / kPermTile, jj = e - v * kPermTile;
    if (jj < rows && v < nv) {
      double* y = it.Y + j0 + jj + it.ldy * v;
      const double z = it.alpha == 0.0 ? 0.0 : it.alpha * tile[jj * LD + v];
      *y = it.beta == 0.0 ? z : z + it.beta * *y;
    }
  }
}

hipError_t launch_batch_permute(const BatchItem* items, const int32_t* tile_op, const int32_t* tile_j0,
                                int64_t ntiles, const int32_t* pinv, double* ws, int nvp, bool out, hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  const dim3 g((unsigned)ntiles), b(256);
#define H2_BP(NVP)                                                                                            \
  do {                                                                                                        \
    if (out) hipLaunchKernelGGL(k_batch_permute_out<NVP>, g, b, 0, s, items, tile_op, tile_j0, pinv, ws);     \
    else hipLaunchKernelGGL(k_batch_permute_in<NVP>, g, b, 0, s, items, tile_op, tile_j0, pinv, ws);          \
  } while (0)
  switch (nvp) {
    case 16: H2_BP(16); break;
    case 32: H2_BP(32); break;
    case 48: H2_BP(48); break;
    case 64: H2_BP(64); break;
    default: return hipErrorInvalidValue;
  }
#undef H2_BP
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// BF16 low-rank path: v_mfma_f32_16x16x32_bf16 (A[i][k] at lane i + 16*(k/8),
// element k%8 of the lane's 8-vector; B[k][j] at lane j + 16*(k/8); C as in
// the FP32 16x16x4 form), FP32 accumulation.  The BF16 copy stores every
// row's matrix row-major (same offsets as the FP64 array, transposed within
// the row), so a lane's eight consecutive k are one 16-byte load.  The input
// is either an FP64 row-major [row][NVP] buffer (the permuted X, the
// downsweep tree y^) or the BF16 column-major [vector][ldb] tree x^ that the
// upsweep launches of this path write (OUT16): x^ is rounded to BF16 once,
// where it is produced, which is the rounding it gets when staged anyway.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
enum { BSRC_F64_RM = 0, BSRC_BF16_CM = 1 };

template <int NT, int MAXT, int BSRC, bool OUT16>
__global__ __launch_bounds__(kT) void k_rows_mfma_bf16(const RowDesc* __restrict__ rows, int64_t nrows,
                                                       const int32_t* __restrict__ colend,
                                                       const int64_t* __restrict__ in_off,
                                                       const __bf16* __restrict__ data, const void* in,
                                                       int64_t ldb, void* out, int64_t ldo, int mode,
                                                       int remap) {
  constexpr int NVP = 16 * NT;
  constexpr int KC = 64;       // columns per LDS chunk (two k-steps of 32)
  constexpr int KCP = KC + 8;  // padded LDS row: 144 bytes, so 16 rows hit 16 distinct 16-byte bank groups
  __shared__ __align__(16) __bf16 bs[NVP * KCP];  // [vector][column]
  __shared__ int32_t s_end[kNbMax];
  __shared__ int64_t s_in[kNbMax];
  __shared__ int64_t s_src[KC];
  // rows by workgroup: plain grid-stride, or (remap) each XCD (workgroups
  // b with the same b % 8) takes one contiguous eighth of the rows, so that
  // neighbouring rows, which share input segments, meet in the same L2
  const int64_t per = remap ? (nrows + 7) / 8 : nrows;
  const int64_t xcd = remap ? blockIdx.x % 8 : 0;
  const int64_t step = remap ? gridDim.x / 8 : gridDim.x;
  for (int64_t jr = remap ? blockIdx.x / 8 : blockIdx.x; jr < per; jr += step) {
    const int64_t ri = xcd * per + jr;
    if (ri >= nrows) break;
    __syncthreads();
    const RowDesc R = rows[ri];
    const int m = R.nrows;
    if (m <= 0) continue;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nb = R.blk_end - R.blk_begin;
    for (int i = tid; i < nb; i += kT) {
      s_end[i] = colend[R.blk_begin + i];
      s_in[i] = in_off[R.blk_begin + i];
    }
    __syncthreads();
    const int ncols = nb > 0 ? s_end[nb - 1] : 0;
    const int mt = (m + 15) >> 4;
    const bool vec = (ncols % 8 == 0) && (R.data_off % 8 == 0);
    f4 acc[MAXT][NT];
#pragma unroll
    for (int i = 0; i < MAXT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = f4{0, 0, 0, 0};
    const int arow = lane & 15, kg = lane >> 4;
    const __bf16* M = data + R.data_off;
    for (int c0 = 0; c0 < ncols; c0 += KC) {
      const int cn = min(KC, ncols - c0);
      // this chunk's A fragments first, so that their loads are in flight
      // while the input is staged
      bf8 a[MAXT][2];
#pragma unroll
      for (int ti = 0; ti < MAXT; ++ti) {
        const int tile = wave + 4 * ti;
        const int r = tile * 16 + arow;
        const bool rok = tile < mt && r < m;
#pragma unroll
        for (int st = 0; st < 2; ++st) {
          const int col = 32 * st + 8 * kg;
          if (rok && vec && col + 8 <= cn) {
            a[ti][st] = __builtin_nontemporal_load(reinterpret_cast<const bf8*>(M + (int64_t)r * ncols + c0 + col));
          } else {
#pragma unroll
            for (int e2 = 0; e2 < 8; ++e2)
              a[ti][st][e2] = (rok && col + e2 < cn) ? M[(int64_t)r * ncols + c0 + col + e2] : (__bf16)0.0f;
          }
        }
      }
      if (c0 > 0) __syncthreads();  // previous chunk's LDS reads done
      if (tid < cn) {
        const int col = c0 + tid;
        int lo = 0, hi = nb - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (s_end[mid] > col) hi = mid; else lo = mid + 1;
        }
        s_src[tid] = s_in[lo] + (col - (lo > 0 ? s_end[lo - 1] : 0));
      }
      __syncthreads();
      if (BSRC == BSRC_BF16_CM) {
        // 8 lanes cover one vector's 64 chunk columns (128 contiguous bytes
        // when the columns are one aligned run of source rows)
        const __bf16* src = static_cast<const __bf16*>(in);
        for (int t = tid; t < NVP * (KC / 8); t += kT) {
          const int g = t & 7, v = t >> 3, j0 = 8 * g;
          const __bf16* sv = src + (int64_t)v * ldb;
          bf8 val;
          if (j0 + 8 <= cn && s_src[j0 + 7] == s_src[j0] + 7 && (s_src[j0] & 7) == 0) {
            val = *reinterpret_cast<const bf8*>(sv + s_src[j0]);
          } else {
#pragma unroll
            for (int e2 = 0; e2 < 8; ++e2) val[e2] = j0 + e2 < cn ? sv[s_src[j0 + e2]] : (__bf16)0.0f;
          }
          *reinterpret_cast<bf8*>(bs + v * KCP + j0) = val;
        }
      } else {
        // consecutive lanes read consecutive vectors of one source row
        const double* src = static_cast<const double*>(in);
        for (int t = tid; t < NVP * (KC / 8); t += kT) {
          const int v = t % NVP, j0 = 8 * (t / NVP);
          bf8 val;
#pragma unroll
          for (int e2 = 0; e2 < 8; ++e2)
            val[e2] = j0 + e2 < cn ? (__bf16)(float)src[s_src[j0 + e2] * NVP + v] : (__bf16)0.0f;
          *reinterpret_cast<bf8*>(bs + v * KCP + j0) = val;
        }
      }
      __syncthreads();
      const int nsteps = (cn + 31) >> 5;
#pragma unroll
      for (int ti = 0; ti < MAXT; ++ti) {
        const int tile = wave + 4 * ti;
        if (tile >= mt) break;
#pragma unroll
        for (int st = 0; st < 2; ++st) {
          if (st >= nsteps) break;
          const int col = 32 * st + 8 * kg;
#pragma unroll
          for (int j = 0; j < NT; ++j) {
            const bf8 b = *reinterpret_cast<const bf8*>(bs + (16 * j + arow) * KCP + col);
            acc[ti][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ti][st], b, acc[ti][j], 0, 0, 0);
          }
        }
      }
    }
#pragma unroll
    for (int ti = 0; ti < MAXT; ++ti) {
      const int tile = wave + 4 * ti;
      if (tile >= mt) break;
#pragma unroll
      for (int j = 0; j < NT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a = tile * 16 + 4 * kg + r;
          if (a < m) {
            if (OUT16) {
              static_cast<__bf16*>(out)[(int64_t)(16 * j + arow) * ldo + R.out_off + a] = (__bf16)acc[ti][j][r];
            } else {
              double* o = static_cast<double*>(out) + (R.out_off + a) * NVP + 16 * j + arow;
              if (mode == MODE_STORE) *o = (double)acc[ti][j][r];
              else *o += (double)acc[ti][j][r];
            }
          }
        }
    }
  }
}

// BF16 copy of the rows' matrices: FP64 column-major m x ncols at data_off
// becomes BF16 row-major at the same offset (rounded through FP32).
__global__ void k_rows_to_bf16(const RowDesc* __restrict__ rows, const int32_t* __restrict__ colend,
                               const double* __restrict__ src, __bf16* __restrict__ dst) {
  const RowDesc R = rows[blockIdx.x];
  const int m = R.nrows;
  const int ncols = R.blk_end > R.blk_begin ? colend[R.blk_end - 1] : 0;
  const int64_t total = (int64_t)m * ncols;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int64_t a = e / ncols, j = e - a * ncols;  // row-major destination index e
    dst[R.data_off + e] = (__bf16)(float)src[R.data_off + a + (int64_t)m * j];
  }
}

// Reduced-precision copy of FP64 data (round to nearest).
__global__ void k_to_f32(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (float)src[e];
}

hipError_t launch_rows_mfma_bf16(const RowDesc* rows, int64_t nrows, const int32_t* colend, const int64_t* in_off,
                                 const void* data, const void* in, bool in16, int64_t ldb, void* out, bool out16,
                                 int64_t ldo, int nvp, int mode, int max_rows, hipStream_t s, int64_t grid,
                                 int remap) {
  if (nrows == 0) return hipSuccess;
  if (out16 && mode != MODE_STORE) return hipErrorInvalidValue;
  if ((in16 || out16) && (ldb % 8 != 0 || ldo % 8 != 0)) return hipErrorInvalidValue;
  const dim3 g((unsigned)grid_of_rows(nrows, grid, remap)), block(kT);
  const __bf16* d = static_cast<const __bf16*>(data);
#define H2_BF4(NT, MAXT, BS, O16) \
  hipLaunchKernelGGL((k_rows_mfma_bf16<NT, MAXT, BS, O16>), g, block, 0, s, rows, nrows, colend, in_off, d, in, \
                     ldb, out, ldo, mode, remap)
#define H2_BF2(NT, MAXT)                                              \
  do {                                                                \
    if (in16) {                                                       \
      if (out16) H2_BF4(NT, MAXT, BSRC_BF16_CM, true);                \
      else H2_BF4(NT, MAXT, BSRC_BF16_CM, false);                     \
    } else {                                                          \
      if (out16) H2_BF4(NT, MAXT, BSRC_F64_RM, true);                 \
      else H2_BF4(NT, MAXT, BSRC_F64_RM, false);                      \
    }                                                                 \
  } while (0)
#define H2_BF(NT)                         \
  do {                                    \
    if (max_rows <= 64) H2_BF2(NT, 1);    \
    else H2_BF2(NT, 4);                   \
  } while (0)
  switch (nvp) {
    case 16: H2_BF(1); break;
    case 32: H2_BF(2); break;
    case 48: H2_BF(3); break;
    case 64: H2_BF(4); break;
    default: return hipErrorInvalidValue;
  }
#undef H2_BF
#undef H2_BF2
#undef H2_BF4
  return hipGetLastError();
}

hipError_t launch_rows_to_bf16(const RowDesc* rows, int64_t nrows, const int32_t* colend, const double* src,
                               void* dst, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_to_bf16, dim3((unsigned)nrows), dim3(256), 0, s, rows, colend, src,
                     static_cast<__bf16*>(dst));
  return hipGetLastError();
}

hipError_t launch_to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32, dim3(4096), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_permute_in_rm(const double* X, int64_t ldx, const int32_t* pinv, double* xt, int64_t n, int nv,
                                int nvp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (nvp > kPassVectorsMfma || nv > nvp) return hipErrorInvalidValue;
  const dim3 g(grid1d(n, kPermTile)), b(256);
  switch (nvp) {
    case 16: hipLaunchKernelGGL(k_permute_in_rm<16>, g, b, 0, s, X, ldx, pinv, xt, n, nv); break;
    case 32: hipLaunchKernelGGL(k_permute_in_rm<32>, g, b, 0, s, X, ldx, pinv, xt, n, nv); break;
    case 48: hipLaunchKernelGGL(k_permute_in_rm<48>, g, b, 0, s, X, ldx, pinv, xt, n, nv); break;
    case 64: hipLaunchKernelGGL(k_permute_in_rm<64>, g, b, 0, s, X, ldx, pinv, xt, n, nv); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_permute_out_rm(const double* Z, const int32_t* pinv, double alpha, double beta, double* Y,
                                 int64_t ldy, int64_t n, int nv, int nvp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (nvp > kPassVectorsMfma || nv > nvp) return hipErrorInvalidValue;
  const dim3 g(grid1d(n, kPermTile)), b(256);
  switch (nvp) {
    case 16: hipLaunchKernelGGL(k_permute_out_rm<16>, g, b, 0, s, Z, pinv, alpha, beta, Y, ldy, n, nv); break;
    case 32: hipLaunchKernelGGL(k_permute_out_rm<32>, g, b, 0, s, Z, pinv, alpha, beta, Y, ldy, n, nv); break;
    case 48: hipLaunchKernelGGL(k_permute_out_rm<48>, g, b, 0, s, Z, pinv, alpha, beta, Y, ldy, n, nv); break;
    case 64: hipLaunchKernelGGL(k_permute_out_rm<64>, g, b, 0, s, Z, pinv, alpha, beta, Y, ldy, n, nv); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rows_wide(const RowDesc* rows, int64_t nrows, const int32_t* colend, const int64_t* in_off,
                            const double* data, const double* in, double* out, int nv, hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_wide, dim3((unsigned)nrows), dim3(kT), 0, s, rows, colend, in_off, data, in, out, nv);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const RowDesc* rows, int64_t nrows, const int64_t* bdata, const int32_t* bmr,
                         const int64_t* bin, const T* data, const double* in, double* out, int nv,
                         hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  const dim3 grid((unsigned)nrows), block(kT);
  if (nv <= 1)
    hipLaunchKernelGGL((k_rows_t<T, 1>), grid, block, 0, s, rows, bdata, bmr, bin, data, in, out, nv);
  else if (nv == 2)
    hipLaunchKernelGGL((k_rows_t<T, 2>), grid, block, 0, s, rows, bdata, bmr, bin, data, in, out, nv);
  else if (nv <= 4)
    hipLaunchKernelGGL((k_rows_t<T, 4>), grid, block, 0, s, rows, bdata, bmr, bin, data, in, out, nv);
  else
    return hipErrorInvalidValue;  // callers pass at most kPassVectors vectors
  return hipGetLastError();
}
template hipError_t launch_gather<double>(const RowDesc*, int64_t, const int64_t*, const int32_t*, const int64_t*,
                                          const double*, const double*, double*, int, hipStream_t);
template hipError_t launch_gather<float>(const RowDesc*, int64_t, const int64_t*, const int32_t*, const int64_t*,
                                         const float*, const double*, double*, int, hipStream_t);

}  // namespace h2
