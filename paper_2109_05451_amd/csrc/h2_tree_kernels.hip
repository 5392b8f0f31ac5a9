// Subtree-fused sweeps of the multi-vector path (FP64 and FP32 MFMA).
//
// The upsweep (Algorithm 1: leaf products x^_t = V_t^T x_t, then the transfer
// levels x^_p = sum_c F_c^T x^_c) and the downsweep (Algorithm 6: y^_c +=
// E_c y^_parent level by level, then the leaf expansion U_t y^_t) are chains
// of small dependent products.  Launched level by level they are latency
// bound: every level is a launch, and every row's matrix (a few KB) is one
// workgroup's whole job.  Here one workgroup owns a subtree and runs several
// levels of it, bottom-up or top-down, in one launch: a level's rows are
// independent (one wave per row, no LDS), a barrier separates levels, and
// each level reads what the previous level of the same workgroup wrote.
// The node ranges of a subtree are contiguous on every level (children are
// stored contiguously, in parent order), so a workgroup's rows on a level are
// one range of the level's row list.
//
// Every output sums the same four-column steps, in the same order, with the
// same MFMA instruction and fragment layout as the row kernels of
// h2_kernels.hip (A[i][k] at lane i + 16k, B[k][j] at lane j + 16k, padded
// steps reading zeros): the results are bitwise those of the per-level
// launches.
#include <algorithm>

#include "h2_internal.h"

namespace h2 {
namespace {

constexpr int kT = 256;
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc;
  static __device__ __forceinline__ d4 op(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator element r of lane l: row 4r + l/16, column l%16
  static __device__ __forceinline__ int row(int r, int akk) { return 4 * r + akk; }
};
template <> struct Mfma<float> {
  typedef f4 acc;
  static __device__ __forceinline__ f4 op(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element r of lane l: row 4(l/16) + r, column l%16
  static __device__ __forceinline__ int row(int r, int akk) { return 4 * akk + r; }
};

__device__ __forceinline__ double* pick(int i, double* b0, double* b1, double* b2, double* b3) {
  return i == 0 ? b0 : i == 1 ? b1 : i == 2 ? b2 : b3;
}

// One row on one wave, vector tiles vt0 .. vt0 + NTW - 1 of it: out (m x
// 16NT, row-major rows of 16NT) = M (m x ncols, column-major at
// data + R.data_off) times the input gathered block by block (row
// in_off[b] + j of `in` for column j of block b).  Each lane keeps a cursor
// over the row's blocks; its column grows by four per step.
// The row's block table is colend[b0 .. b0 + nb), in_off[b0 .. b0 + nb):
// the global tables (b0 = R.blk_begin) or a wave's copy in LDS (b0 = 0).
//
// FL: the matrix is read from the row's fragment-ordered copy at
// data + R.fl_off instead (see k_rows_to_fl): the same values reach the same
// MFMA operands, so the result is bitwise the same, but every load of a
// wave reads whole 128-byte lines (two four-column steps per lane, 16 bytes
// for FP64) instead of 16-row pieces of columns that straddle lines.
template <typename T, int NT, int NTW, int MT, bool FL = false>
__device__ __forceinline__ void wave_row(const RowDesc& R, const int32_t* colend, const int64_t* in_off, int b0,
                                         const T* __restrict__ data, const double* in, double* out, int mode,
                                         int lane, int vt0) {
  typedef typename Mfma<T>::acc CT;
  constexpr int NVP = 16 * NT;
  const int m = R.nrows;
  const int nb = R.blk_end - R.blk_begin;
  if (m <= 0) return;
  const int ncols = nb > 0 ? colend[b0 + nb - 1] : 0;
  const int mt = (m + 15) >> 4;
  const int arow = lane & 15, akk = lane >> 4;
  CT acc[MT][NTW];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int j = 0; j < NTW; ++j) acc[i][j] = CT{0, 0, 0, 0};
  int b = b0, bstart = 0;
  int bend = nb > 0 ? colend[b] : 0;
  int64_t boff = nb > 0 ? in_off[b] : 0;
  // fragment order: npair full pairs of four-column steps, each 8m values
  // (full 16-row tiles: 128 values in lane order, two per lane; the last
  // m % 16 rows: 8 (m % 16) values, two per active lane), then the last
  // ncols % 8 columns column-major
  const int npair = FL ? ncols >> 3 : 0;
  const int nfull = m >> 4, rem = m & 15;
  const T* M = data + (FL ? R.fl_off : R.data_off);
  const T* Mt = M + (int64_t)8 * m * npair;
  // four-column steps loaded per iteration: four, or two when the
  // accumulators are many (keeps two waves per SIMD at 64 rows x 64 vectors)
  constexpr int U = MT * NTW > 8 ? 2 : 4;
  for (int c0 = 0; c0 < ncols; c0 += 4 * U) {
    T a[U][MT], bf[U][NTW];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int col = c0 + 4 * u + akk;
      const bool ok = col < ncols;
      if (ok) {
        while (col >= bend) {
          bstart = bend;
          ++b;
          bend = colend[b];
          boff = in_off[b];
        }
      }
      const double* src = in + (boff + (col - bstart)) * NVP + 16 * vt0 + arow;
#pragma unroll
      for (int j = 0; j < NTW; ++j) bf[u][j] = ok ? (T)src[16 * j] : (T)0;
      if (!FL) {
#pragma unroll
        for (int ti = 0; ti < MT; ++ti) {
          const int r = 16 * ti + arow;
          a[u][ti] = (ok && ti < mt && r < m) ? __builtin_nontemporal_load(M + r + (int64_t)m * col) : (T)0;
        }
      }
    }
    if (FL) {
      typedef T t2 __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int u2 = 0; u2 < U / 2; ++u2) {
        const int p = (c0 >> 3) + u2;  // wave-uniform
        if (p < npair) {
          const T* P = M + (int64_t)8 * m * p;
#pragma unroll
          for (int ti = 0; ti < MT; ++ti) {
            t2 v = t2{(T)0, (T)0};
            if (ti < nfull)
              v = __builtin_nontemporal_load(reinterpret_cast<const t2*>(P + 128 * ti + 2 * lane));
            else if (ti == nfull && arow < rem)
              v = __builtin_nontemporal_load(reinterpret_cast<const t2*>(P + 128 * nfull + 2 * (akk * rem + arow)));
            a[2 * u2][ti] = v[0];
            a[2 * u2 + 1][ti] = v[1];
          }
        } else {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int col = c0 + 8 * u2 + 4 * h + akk;
            const bool ok = col < ncols;
#pragma unroll
            for (int ti = 0; ti < MT; ++ti) {
              const int r = 16 * ti + arow;
              a[2 * u2 + h][ti] = (ok && ti < mt && r < m)
                                      ? __builtin_nontemporal_load(Mt + r + (int64_t)m * (col - 8 * npair))
                                      : (T)0;
            }
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (c0 + 4 * u < ncols) {
#pragma unroll
        for (int ti = 0; ti < MT; ++ti) {
          if (ti < mt) {
#pragma unroll
            for (int j = 0; j < NTW; ++j) acc[ti][j] = Mfma<T>::op(a[u][ti], bf[u][j], acc[ti][j]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int ti = 0; ti < MT; ++ti) {
    if (ti >= mt) break;
#pragma unroll
    for (int j = 0; j < NTW; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a = 16 * ti + Mfma<T>::row(r, akk);
        if (a < m) {
          double* o = out + (R.out_off + a) * NVP + 16 * (vt0 + j) + arow;
          if (mode == MODE_STORE) *o = (double)acc[ti][j][r];
          else *o += (double)acc[ti][j][r];
        }
      }
  }
}

// One launch of a fused sweep: workgroup w takes, for each of the group's
// levels in order, the rows ranges[w * nlev + lev] of the row table.  A row
// is computed by NT / NTW waves, each with NTW of its vector tiles (two waves
// per row when one wave's accumulators would leave one wave per SIMD), so
// the four waves hold 4 NTW / NT rows at a time.  Buffers: 0 X~, 1 x^, 2 y^,
// 3 the leaf-expansion output.
template <typename T, int NT, int NTW, int MT>
__global__ __launch_bounds__(kT) void k_tree(const int2* __restrict__ ranges, TreeLevels L,
                                             const RowDesc* __restrict__ rows, const int32_t* __restrict__ colend,
                                             const int64_t* __restrict__ in_off, const T* __restrict__ data,
                                             double* b0, double* b1, double* b2, double* b3) {
  constexpr int WPR = NT / NTW, RPW = 4 / WPR;  // waves per row, rows per workgroup at a time
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int slot = wave / WPR, vt0 = (wave % WPR) * NTW;
  for (int lev = 0; lev < L.nlev; ++lev) {
    if (lev > 0) __syncthreads();  // the previous level's outputs are this level's inputs
    const int2 rr = ranges[(int64_t)blockIdx.x * L.nlev + lev];
    const double* in = pick(L.in[lev], b0, b1, b2, b3);
    double* out = pick(L.out[lev], b0, b1, b2, b3);
    for (int ri = rr.x + slot; ri < rr.y; ri += RPW) {
      const RowDesc R = rows[ri];
      wave_row<T, NT, NTW, MT>(R, colend, in_off, R.blk_begin, data, in, out, L.mode[lev], lane, vt0);
    }
  }
}

// A plain row list with the same wave-per-row product: workgroup b holds
// 4 NTW / NT rows at a time, rows taken grid-stride.  One more form of the
// multi-vector row launches for the tuner: no barriers, the matrix and input
// fragments read straight from memory, many rows in flight per CU.  Each
// wave copies its row's block table into its own LDS region first, so the
// column cursor (one step per block, dozens of blocks in a coupling or dense
// row) reads LDS instead of waiting on dependent global loads.
// OCC > 1: compiled for at least OCC waves per SIMD (the register budget
// shrinks from 128 to 96 at OCC 5, with a few registers spilled): more rows'
// loads in flight per CU for launches bound by memory latency.
template <typename T, int NT, int NTW, int MT, bool FL, int OCC>
__global__ __launch_bounds__(kT, OCC) void k_wave_rows(const RowDesc* __restrict__ rows, int64_t nrows,
                                                  const int32_t* __restrict__ colend,
                                                  const int64_t* __restrict__ in_off, const T* __restrict__ data,
                                                  const double* in, double* out, int mode, int remap) {
  constexpr int WPR = NT / NTW, RPW = 4 / WPR;
  __shared__ int32_t s_end[4][kNbMax];
  __shared__ int64_t s_in[4][kNbMax];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int slot = wave / WPR, vt0 = (wave % WPR) * NTW;
  // rows by workgroup: grid-stride, or (remap; a grid of a multiple of 8)
  // each XCD (workgroups b with the same b % 8) takes one contiguous eighth
  // of the rows, so that rows in flight together on an XCD are neighbours in
  // the row order and their shared input segments meet in that XCD's L2
  const int64_t per = remap ? (nrows + 7) / 8 : nrows;
  const int64_t base = remap ? (int64_t)(blockIdx.x % 8) * per : 0;
  const int64_t wg = remap ? blockIdx.x / 8 : blockIdx.x;
  const int64_t nwg = remap ? gridDim.x / 8 : gridDim.x;
  for (int64_t jr = wg * RPW + slot; jr < per; jr += nwg * RPW) {
    const int64_t ri = base + jr;
    if (ri >= nrows) break;
    const RowDesc R = rows[ri];
    const int nb = R.blk_end - R.blk_begin;  // <= kNbMax for rows of these tables
    __builtin_amdgcn_wave_barrier();         // the previous row's table fully read
    for (int i = lane; i < nb; i += 64) {
      s_end[wave][i] = colend[R.blk_begin + i];
      s_in[wave][i] = in_off[R.blk_begin + i];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    wave_row<T, NT, NTW, MT, FL>(R, s_end[wave], s_in[wave], 0, data, in, out, mode, lane, vt0);
  }
}

// The fragment-ordered copy of each row (one workgroup per row,
// grid-stride): dst[R.fl_off + e], e < m * ncols, from the column-major
// src[R.data_off + r + m * c].  For e < 8 m npair (npair = ncols / 8): pair
// p = e / 8m of four-column steps; within it, full row tile t, lane l
// (row 16 t + l % 16, step column l / 16) and step u at 128 t + 2 l + u,
// then the last rem = m % 16 rows, lane i + 16 k (i < rem) at
// 128 (m / 16) + 2 (k rem + i) + u; the column is 8 p + 4 u + k.  The last
// ncols % 8 columns follow column-major.
template <typename T>
__global__ __launch_bounds__(256) void k_rows_to_fl(const RowDesc* __restrict__ rows, int64_t nrows,
                                                    const int32_t* __restrict__ colend, const T* __restrict__ src,
                                                    T* __restrict__ dst) {
  for (int64_t ri = blockIdx.x; ri < nrows; ri += gridDim.x) {
    const RowDesc R = rows[ri];
    const int m = R.nrows, nb = R.blk_end - R.blk_begin;
    const int ncols = nb > 0 ? colend[R.blk_end - 1] : 0;
    const int64_t npair = ncols >> 3, body = (int64_t)8 * m * npair, total = (int64_t)m * ncols;
    const int nfull = m >> 4, rem = m & 15;
    for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
      int64_t r, c;
      if (e < body) {
        const int64_t p = e / (8 * m);
        const int x = (int)(e - p * 8 * m);
        int u, k, i;
        if (x < 128 * nfull) {
          const int t = x >> 7, y = x & 127, l = y >> 1;
          u = y & 1; k = l >> 4; i = 16 * t + (l & 15);
        } else {
          const int y = x - 128 * nfull, l = y >> 1;
          u = y & 1; k = l / rem; i = 16 * nfull + l % rem;
        }
        r = i;
        c = 8 * p + 4 * u + k;
      } else {
        const int64_t t = e - body;
        r = t % m;
        c = 8 * npair + t / m;
      }
      dst[R.fl_off + e] = src[R.data_off + r + (int64_t)m * c];
    }
  }
}

// Y[j, v] = alpha * (Z[pinv[j], v] + Z2[pinv[j], v]) + beta * Y[j, v]: the
// dense partial plus the leaf expansion (row-major NVP, tree order) into the
// caller's column-major Y, through an LDS tile of 64 points so that both
// sides are accessed with coalesced loads and stores.
template <int NVP>
__global__ __launch_bounds__(256) void k_permute_out_rm2(const double* __restrict__ Z, const double* __restrict__ Z2,
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
    if (jj < rows && v < nv) {
      const int64_t src = (int64_t)pinv[j0 + jj] * NVP + v;
      r[i] = __builtin_nontemporal_load(Z + src) + __builtin_nontemporal_load(Z2 + src);
    } else {
      r[i] = 0.0;
    }
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

}  // namespace

hipError_t launch_permute_out_rm2(const double* Z, const double* Z2, const int32_t* pinv, double alpha, double beta,
                                  double* Y, int64_t ldy, int64_t n, int nv, int nvp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (nvp > kPassVectorsMfma || nv > nvp) return hipErrorInvalidValue;
  const dim3 g((unsigned)((n + kPermTile - 1) / kPermTile)), b(256);
  switch (nvp) {
    case 16: hipLaunchKernelGGL(k_permute_out_rm2<16>, g, b, 0, s, Z, Z2, pinv, alpha, beta, Y, ldy, n, nv); break;
    case 32: hipLaunchKernelGGL(k_permute_out_rm2<32>, g, b, 0, s, Z, Z2, pinv, alpha, beta, Y, ldy, n, nv); break;
    case 48: hipLaunchKernelGGL(k_permute_out_rm2<48>, g, b, 0, s, Z, Z2, pinv, alpha, beta, Y, ldy, n, nv); break;
    case 64: hipLaunchKernelGGL(k_permute_out_rm2<64>, g, b, 0, s, Z, Z2, pinv, alpha, beta, Y, ldy, n, nv); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Workgroups of a wave-row launch of rpw rows per workgroup pass: enough
// for every row at once, or `grid`; with the XCD remap a multiple of 8
// covering eight equal row ranges.
inline int64_t wave_grid(int64_t nrows, int rpw, int64_t grid, int remap) {
  if (!remap) {
    const int64_t need = (nrows + rpw - 1) / rpw;
    return grid > 0 && grid < need ? grid : need;
  }
  const int64_t per = (nrows + 7) / 8, needx = (per + rpw - 1) / rpw;
  return grid > 0 ? std::min<int64_t>((grid + 7) / 8 * 8, 8 * needx) : 8 * needx;
}

template <typename T>
hipError_t launch_rows_to_fl(const RowDesc* rows, int64_t nrows, const int32_t* colend, const T* src, T* dst,
                             hipStream_t s) {
  if (nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_to_fl<T>, dim3((unsigned)std::min<int64_t>(nrows, 65536)), dim3(256), 0, s, rows, nrows,
                     colend, src, dst);
  return hipGetLastError();
}
template hipError_t launch_rows_to_fl<double>(const RowDesc*, int64_t, const int32_t*, const double*, double*,
                                              hipStream_t);
template hipError_t launch_rows_to_fl<float>(const RowDesc*, int64_t, const int32_t*, const float*, float*,
                                             hipStream_t);

template <typename T>
hipError_t launch_wave_rows(const RowDesc* rows, int64_t nrows, const int32_t* colend, const int64_t* in_off,
                            const T* data, const double* in, double* out, int nvp, int mode, int max_rows,
                            hipStream_t s, int64_t grid, bool narrow, int remap, const T* fl, int occ) {
  if (nrows == 0) return hipSuccess;
  if (max_rows > 64) return hipErrorInvalidValue;
  // narrow: a wave per 16-vector tile (NT waves per row, more waves resident); else a wave per row, or
  // two when one wave's accumulators would leave a single wave per SIMD
#define H2_WR_K(NT, NTW, MT, G)                                                                          \
  do {                                                                                                   \
    constexpr bool HI = NTW == 1 && MT <= 3;  /* forms that fit 96 registers with little spilling */     \
    if (fl && occ == 5 && HI)                                                                            \
      hipLaunchKernelGGL((k_wave_rows<T, NT, NTW, MT, true, HI ? 5 : 1>), G, dim3(kT), 0, s, rows, nrows, \
                         colend, in_off, fl, in, out, mode, remap);                                      \
    else if (occ == 5 && HI)                                                                             \
      hipLaunchKernelGGL((k_wave_rows<T, NT, NTW, MT, false, HI ? 5 : 1>), G, dim3(kT), 0, s, rows, nrows, \
                         colend, in_off, data, in, out, mode, remap);                                    \
    else if (fl)                                                                                         \
      hipLaunchKernelGGL((k_wave_rows<T, NT, NTW, MT, true, 1>), G, dim3(kT), 0, s, rows, nrows, colend, in_off, \
                         fl, in, out, mode, remap);                                                      \
    else                                                                                                 \
      hipLaunchKernelGGL((k_wave_rows<T, NT, NTW, MT, false, 1>), G, dim3(kT), 0, s, rows, nrows, colend, \
                         in_off, data, in, out, mode, remap);                                            \
  } while (0)
#define H2_WR(NT, MT)                                                                                    \
  do {                                                                                                   \
    if (narrow && (NT == 2 || NT == 4)) {                                                                \
      constexpr int RPWN = 4 / NT;                                                                       \
      H2_WR_K(NT, 1, MT, dim3((unsigned)wave_grid(nrows, RPWN, grid, remap)));                           \
      break;                                                                                             \
    }                                                                                                    \
    constexpr int NTW = (MT * NT > 8 && NT % 2 == 0) ? NT / 2 : NT, RPW = 4 / (NT / NTW);               \
    H2_WR_K(NT, NTW, MT, dim3((unsigned)wave_grid(nrows, RPW, grid, remap)));                           \
  } while (0)
#define H2_WR_NT(NT)                          \
  do {                                        \
    if (max_rows <= 16) H2_WR(NT, 1);         \
    else if (max_rows <= 32) H2_WR(NT, 2);    \
    else if (max_rows <= 48) H2_WR(NT, 3);    \
    else H2_WR(NT, 4);                        \
  } while (0)
  switch (nvp) {
    case 16: H2_WR_NT(1); break;
    case 32: H2_WR_NT(2); break;
    case 48: H2_WR_NT(3); break;
    case 64: H2_WR_NT(4); break;
    default: return hipErrorInvalidValue;
  }
#undef H2_WR_NT
#undef H2_WR
#undef H2_WR_K
  return hipGetLastError();
}
template hipError_t launch_wave_rows<double>(const RowDesc*, int64_t, const int32_t*, const int64_t*, const double*,
                                             const double*, double*, int, int, int, hipStream_t, int64_t, bool, int,
                                             const double*, int);
template hipError_t launch_wave_rows<float>(const RowDesc*, int64_t, const int32_t*, const int64_t*, const float*,
                                            const double*, double*, int, int, int, hipStream_t, int64_t, bool, int,
                                            const float*, int);

template <typename T>
hipError_t launch_tree(const int2* ranges, int64_t nwg, const TreeLevels& L, const RowDesc* rows,
                       const int32_t* colend, const int64_t* in_off, const T* data, double* const bufs[4], int nvp,
                       int max_rows, hipStream_t s) {
  if (nwg == 0 || L.nlev == 0) return hipSuccess;
  if (L.nlev > kMaxTreeLevels || max_rows > 64) return hipErrorInvalidValue;
  const dim3 g((unsigned)nwg), b(kT);
#define H2_TREE(NT, MT)                                                                                      \
  hipLaunchKernelGGL((k_tree<T, NT, (MT * NT > 8 && NT % 2 == 0 ? NT / 2 : NT), MT>), g, b, 0, s, ranges, L, rows, \
                     colend, in_off, data, bufs[0], bufs[1], bufs[2], bufs[3])
#define H2_TREE_NT(NT)                   \
  do {                                   \
    if (max_rows <= 16) H2_TREE(NT, 1);  \
    else if (max_rows <= 32) H2_TREE(NT, 2); \
    else if (max_rows <= 48) H2_TREE(NT, 3); \
    else H2_TREE(NT, 4);                 \
  } while (0)
  switch (nvp) {
    case 16: H2_TREE_NT(1); break;
    case 32: H2_TREE_NT(2); break;
    case 48: H2_TREE_NT(3); break;
    case 64: H2_TREE_NT(4); break;
    default: return hipErrorInvalidValue;
  }
#undef H2_TREE_NT
#undef H2_TREE
  return hipGetLastError();
}
template hipError_t launch_tree<double>(const int2*, int64_t, const TreeLevels&, const RowDesc*, const int32_t*,
                                        const int64_t*, const double*, double* const[4], int, int, hipStream_t);
template hipError_t launch_tree<float>(const int2*, int64_t, const TreeLevels&, const RowDesc*, const int32_t*,
                                       const int64_t*, const float*, double* const[4], int, int, hipStream_t);

}  // namespace h2
