// HIP kernels of the H^2 matrix-vector product for CDNA4 (gfx950).
//
// Vector trees x^ and y^ (Section 3: one k-vector per node and vector) live
// in an H x nv column-major array; node c's entries are rows
// [hoff[c], hoff[c] + k).  The tree-ordered input copy and the dense-phase
// output are n x nv column-major.  Every output entry is produced by exactly
// one thread with a fixed summation order: no atomics, bitwise-reproducible
// results.
#include "h2_internal.h"

namespace h2 {
namespace {

constexpr int kRowThreads = 256;
constexpr int kSmallThreads = 64;

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

// Leaf products x^_t = B_t^T x~_t (Algorithm 1, first batched product).
// One workgroup per leaf; B_t is m x k column-major at B + lo*k.
__global__ void k_leaf_up(const double* __restrict__ B, int k, int64_t leaf0, const int32_t* __restrict__ lo,
                          const int32_t* __restrict__ msz, const int64_t* __restrict__ hoff,
                          const double* __restrict__ xt, int64_t n, double* __restrict__ xh, int64_t H, int nv) {
  const int64_t t = leaf0 + blockIdx.x;
  const int l0 = lo[t], m = msz[t];
  const double* Bt = B + (int64_t)l0 * k;
  for (int o = threadIdx.x; o < k * nv; o += blockDim.x) {
    const int a = o % k, v = o / k;
    const double* x = xt + l0 + n * v;
    const double* col = Bt + (int64_t)m * a;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s += col[i] * x[i];
    xh[hoff[t] + a + H * v] = s;
  }
}

// Transfer upsweep of one level (Algorithm 1, the loop over levels):
// x^_p = sum over children c of T_c^T x^_c, T_c is kc x kp column-major.
// One workgroup per parent; the parent owns its sum, so no atomics.
__global__ void k_transfer_up(const double* __restrict__ T, int kc, int kp, int64_t pbegin, int64_t cbegin,
                              const int32_t* __restrict__ cptr, const int64_t* __restrict__ hoff,
                              double* __restrict__ xh, int64_t H, int nv) {
  const int64_t p = pbegin + blockIdx.x;
  const int c0 = cptr[p], c1 = cptr[p + 1];
  for (int o = threadIdx.x; o < kp * nv; o += blockDim.x) {
    const int b = o % kp, v = o / kp;
    double s = 0.0;
    for (int c = c0; c < c1; ++c) {
      const double* col = T + (int64_t)(c - cbegin) * kc * kp + (int64_t)kc * b;
      const double* x = xh + hoff[c] + H * v;
      for (int a = 0; a < kc; ++a) s += col[a] * x[a];
    }
    xh[hoff[p] + b + H * v] = s;
  }
}

// Transfer downsweep of one level (Algorithm 6): y^_c += T_c y^_parent.
__global__ void k_transfer_down(const double* __restrict__ T, int kc, int kp, int64_t cbegin,
                                const int32_t* __restrict__ parent, const int64_t* __restrict__ hoff,
                                double* __restrict__ yh, int64_t H, int nv) {
  const int64_t c = cbegin + blockIdx.x;
  const int p = parent[c];
  const double* Tc = T + (int64_t)blockIdx.x * kc * kp;
  for (int o = threadIdx.x; o < kc * nv; o += blockDim.x) {
    const int a = o % kc, v = o / kc;
    const double* y = yh + hoff[p] + H * v;
    double s = 0.0;
    for (int b = 0; b < kp; ++b) s += Tc[a + (int64_t)kc * b] * y[b];
    yh[hoff[c] + a + H * v] += s;
  }
}

// Leaf expansion and output (Algorithm 6, last product), fused with the
// dense-phase partial and the BLAS update, written in original order:
// Y[perm[lo+i], v] = alpha * (zn[lo+i, v] + (B_t y^_t)[i, v]) + beta * Y[...].
__global__ void k_leaf_down(const double* __restrict__ B, int k, int64_t leaf0, const int32_t* __restrict__ lo,
                            const int32_t* __restrict__ msz, const int64_t* __restrict__ hoff,
                            const double* __restrict__ yh, int64_t H, const double* __restrict__ zn, int64_t n,
                            const int32_t* __restrict__ perm, double alpha, double beta, double* __restrict__ Y,
                            int64_t ldy, int nv) {
  const int64_t t = leaf0 + blockIdx.x;
  const int l0 = lo[t], m = msz[t];
  const double* Bt = B + (int64_t)l0 * k;
  for (int o = threadIdx.x; o < m * nv; o += blockDim.x) {
    const int i = o % m, v = o / m;
    const double* y = yh + hoff[t] + H * v;
    double s = zn[l0 + i + n * v];
    for (int a = 0; a < k; ++a) s += Bt[i + (int64_t)m * a] * y[a];
    double* yo = Y + perm[l0 + i] + ldy * v;
    *yo = beta == 0.0 ? alpha * s : alpha * s + beta * *yo;
  }
}

// Block-row streaming product, for the coupling blocks of all levels at once
// (Algorithm 4: the levels are independent) and for the dense leaf blocks.
// The blocks of a row are contiguous and together form a column-major
// nrows x ncols matrix M; out[:, v] = M * in_gathered[:, v].  Thread
// (a, g) owns row a and columns g, g+G, g+2G, ...: consecutive threads read
// consecutive addresses, so the workgroup streams M with coalesced loads.
// Partial sums over g are combined in LDS in a fixed order.
template <int NVB>
__global__ __launch_bounds__(kRowThreads) void k_stream_rows(
    const RowDesc* __restrict__ rows, const int32_t* __restrict__ colend, const int64_t* __restrict__ in_off,
    const double* __restrict__ data, const double* __restrict__ in, double* __restrict__ out, int nv) {
  __shared__ double red[kRowThreads * NVB];
  const RowDesc R = rows[blockIdx.x];
  const int m = R.nrows;
  if (m <= 0) return;
  const int tid = threadIdx.x;
  const int G = kRowThreads / m;
  const int a = tid % m, g = tid / m;
  const int nb = R.blk_end - R.blk_begin;
  const int ncols = nb > 0 ? colend[R.blk_end - 1] : 0;
  const double* M = data + R.data_off;
  for (int v0 = 0; v0 < nv; v0 += NVB) {
    const int nvb = min(NVB, nv - v0);
    double acc[NVB];
#pragma unroll
    for (int v = 0; v < NVB; ++v) acc[v] = 0.0;
    if (g < G && nb > 0) {
      int b = R.blk_begin, bstart = 0, bend = colend[b];
      for (int j = g; j < ncols; j += G) {
        while (j >= bend) {
          bstart = bend;
          ++b;
          bend = colend[b];
        }
        const double mv = M[(int64_t)a + (int64_t)m * j];
        const double* x = in + in_off[b] + (j - bstart) + R.in_ld * v0;
#pragma unroll
        for (int v = 0; v < NVB; ++v)
          if (v < nvb) acc[v] += mv * x[R.in_ld * v];
      }
    }
    __syncthreads();
    if (g < G) {
#pragma unroll
      for (int v = 0; v < NVB; ++v) red[(g * NVB + v) * m + a] = acc[v];
    }
    __syncthreads();
    for (int o = tid; o < m * nvb; o += kRowThreads) {
      const int aa = o % m, v = o / m;
      double s = 0.0;
      for (int gg = 0; gg < G; ++gg) s += red[(gg * NVB + v) * m + aa];
      out[R.out_off + aa + R.out_ld * (v0 + v)] = s;
    }
  }
}

// Transposed block-column product (op 'T'): out[b, v] = sum over the blocks
// of the column, sum_a Mblk[a, b] in[a, v].  Column b of a stored block is
// contiguous, so each thread streams its own column.
__global__ void k_gather_rows(const RowDesc* __restrict__ rows, const int64_t* __restrict__ bdata,
                              const int32_t* __restrict__ bmr, const int64_t* __restrict__ bin,
                              const double* __restrict__ data, const double* __restrict__ in,
                              double* __restrict__ out, int nv) {
  const RowDesc R = rows[blockIdx.x];
  const int ms = R.nrows;
  for (int o = threadIdx.x; o < ms * nv; o += blockDim.x) {
    const int b = o % ms, v = o / ms;
    double s = 0.0;
    for (int blk = R.blk_begin; blk < R.blk_end; ++blk) {
      const int mr = bmr[blk];
      const double* col = data + bdata[blk] + (int64_t)mr * b;
      const double* x = in + bin[blk] + R.in_ld * v;
      for (int a = 0; a < mr; ++a) s += col[a] * x[a];
    }
    out[R.out_off + b + R.out_ld * v] = s;
  }
}

inline unsigned grid1d(int64_t total, int threads) { return (unsigned)((total + threads - 1) / threads); }

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

hipError_t launch_leaf_up(const double* B, int k, int64_t leaf0, int64_t nleaves, const int32_t* lo,
                          const int32_t* m, const int64_t* hoff, const double* xt, int64_t n, double* xh,
                          int64_t H, int nv, hipStream_t s) {
  if (nleaves == 0 || k == 0) return hipSuccess;
  hipLaunchKernelGGL(k_leaf_up, dim3((unsigned)nleaves), dim3(kSmallThreads), 0, s, B, k, leaf0, lo, m, hoff,
                     xt, n, xh, H, nv);
  return hipGetLastError();
}

hipError_t launch_transfer_up(const double* T, int kc, int kp, int64_t pbegin, int64_t pcount, int64_t cbegin,
                              const int32_t* cptr, const int64_t* hoff, double* xh, int64_t H, int nv,
                              hipStream_t s) {
  if (pcount == 0 || kp == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transfer_up, dim3((unsigned)pcount), dim3(kSmallThreads), 0, s, T, kc, kp, pbegin,
                     cbegin, cptr, hoff, xh, H, nv);
  return hipGetLastError();
}

hipError_t launch_transfer_down(const double* T, int kc, int kp, int64_t cbegin, int64_t ccount,
                                const int32_t* parent, const int64_t* hoff, double* yh, int64_t H, int nv,
                                hipStream_t s) {
  if (ccount == 0 || kc == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transfer_down, dim3((unsigned)ccount), dim3(kSmallThreads), 0, s, T, kc, kp, cbegin,
                     parent, hoff, yh, H, nv);
  return hipGetLastError();
}

hipError_t launch_leaf_down(const double* B, int k, int64_t leaf0, int64_t nleaves, const int32_t* lo,
                            const int32_t* m, const int64_t* hoff, const double* yh, int64_t H, const double* zn,
                            int64_t n, const int32_t* perm, double alpha, double beta, double* Y, int64_t ldy,
                            int nv, hipStream_t s) {
  if (nleaves == 0) return hipSuccess;
  hipLaunchKernelGGL(k_leaf_down, dim3((unsigned)nleaves), dim3(kSmallThreads), 0, s, B, k, leaf0, lo, m, hoff,
                     yh, H, zn, n, perm, alpha, beta, Y, ldy, nv);
  return hipGetLastError();
}

hipError_t launch_stream_rows(const StreamSched& sc, const double* data, const double* in, double* out, int nv,
                              hipStream_t s) {
  const size_t nrows = sc.rows.size();
  if (nrows == 0) return hipSuccess;
  if (nv <= 1) {
    hipLaunchKernelGGL(k_stream_rows<1>, dim3((unsigned)nrows), dim3(kRowThreads), 0, s, sc.d_rows, sc.d_colend,
                       sc.d_in_off, data, in, out, nv);
  } else if (nv <= 4) {
    hipLaunchKernelGGL(k_stream_rows<4>, dim3((unsigned)nrows), dim3(kRowThreads), 0, s, sc.d_rows, sc.d_colend,
                       sc.d_in_off, data, in, out, nv);
  } else {
    hipLaunchKernelGGL(k_stream_rows<8>, dim3((unsigned)nrows), dim3(kRowThreads), 0, s, sc.d_rows, sc.d_colend,
                       sc.d_in_off, data, in, out, nv);
  }
  return hipGetLastError();
}

hipError_t launch_gather_rows(const GatherSched& sc, const double* data, const double* in, double* out, int nv,
                              hipStream_t s) {
  const size_t nrows = sc.rows.size();
  if (nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)nrows), dim3(kRowThreads), 0, s, sc.d_rows, sc.d_data, sc.d_mr,
                     sc.d_in_off, data, in, out, nv);
  return hipGetLastError();
}

}  // namespace h2
