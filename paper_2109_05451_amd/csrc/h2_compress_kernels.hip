// Kernels of the algebraic recompression (Section 5 of the paper), FP64.
//
// Every operation works on small dense matrices (at most 64 columns; the
// QR operands at most 8192 elements), one workgroup per matrix (or per
// output block), with the operands staged in LDS:
//   k_qr       Householder QR with the thin Q formed in place (reflectors
//              applied backwards), R written separately
//   k_gemm     C = beta C + alpha sum_p op(A_p) op(B_p) over a list of pairs
//              (segmented sums such as the Gram matrix of a block row)
//   k_triple   C = beta C + L M R^T (coupling transforms, projections, the
//              Gram downsweep)
//   k_eig      symmetric eigendecomposition by parallel cyclic Jacobi
//              (eigenvalues in descending order, eigenvectors as columns)
// plus small elementwise helpers.  All index bounds come from descriptors
// that the host checks against the allocations before any launch.
#include <hip/hip_runtime.h>

#include "h2_compress.h"

namespace h2 {
namespace {

constexpr int kCT = 256;  // threads per workgroup
constexpr int kTile = 64; // largest output rows / columns of one GEMM task

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Householder QR of an r x c column-major matrix (r * c <= kQrMaxElems).
// Reflector j (j < nr = min(r, c)) is H_j = I - tau_j v_j v_j^T with
// v_j[j] = 1, zeros above j, stored below the diagonal; beta_j = R[j][j].
// Q (r x c): the first nr columns of H_0 ... H_{nr-1}, zero columns after.
// R (c x c): upper triangle of the factored matrix in rows < nr, zero rows
// after (so that A = Q R also when r < c).
__global__ __launch_bounds__(kCT) void k_qr(const QrTask* __restrict__ tasks) {
  __shared__ double sA[kQrMaxElems];
  __shared__ double s_tau[kMaxCompressRank];
  __shared__ double s_scal[2];
  const QrTask T = tasks[blockIdx.x];
  const int r = T.rows, c = T.cols, nr = min(r, c);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < r * c; e += kCT) {
    const int j = e / r, i = e - j * r;
    sA[e] = T.A[i + (int64_t)j * T.lda];
  }
  __syncthreads();
  for (int j = 0; j < nr; ++j) {
    double* col = sA + j * r;
    if (wave == 0) {
      double x2 = 0.0;
      for (int i = j + 1 + lane; i < r; i += 64) x2 += col[i] * col[i];
      x2 = wave_sum(x2);
      if (lane == 0) {
        const double alpha = col[j];
        double tau = 0.0, scal = 0.0, beta = alpha;
        if (x2 > 0.0) {
          const double nrm = sqrt(alpha * alpha + x2);
          beta = alpha >= 0.0 ? -nrm : nrm;
          tau = (beta - alpha) / beta;
          scal = 1.0 / (alpha - beta);
        }
        s_tau[j] = tau;
        s_scal[0] = scal;
        s_scal[1] = beta;
      }
    }
    __syncthreads();
    const double scal = s_scal[0], tau = s_tau[j];
    for (int i = j + 1 + tid; i < r; i += kCT) col[i] *= scal;
    __syncthreads();
    if (tid == 0) col[j] = s_scal[1];
    // apply H_j to columns j+1 .. c-1 (one wave per column)
    if (tau != 0.0) {
      for (int cc = j + 1 + wave; cc < c; cc += kCT / 64) {
        double* a = sA + cc * r;
        double w = 0.0;
        for (int i = j + lane; i < r; i += 64) w += (i == j ? 1.0 : col[i]) * a[i];
        w = wave_sum(w) * tau;
        for (int i = j + lane; i < r; i += 64) a[i] -= w * (i == j ? 1.0 : col[i]);
      }
    }
    __syncthreads();
  }
  // R
  for (int e = tid; e < c * c; e += kCT) {
    const int j = e / c, i = e - j * c;
    T.R[i + (int64_t)j * T.ldr] = (i < nr && i <= j) ? sA[i + j * r] : 0.0;
  }
  __syncthreads();
  // thin Q in place, reflectors taken backwards
  for (int j = nr - 1; j >= 0; --j) {
    double* col = sA + j * r;
    const double tau = s_tau[j];
    // H_j on columns j+1 .. nr-1 (their rows above j are zero, so only rows >= j change)
    if (tau != 0.0) {
      for (int cc = j + 1 + wave; cc < nr; cc += kCT / 64) {
        double* a = sA + cc * r;
        double w = 0.0;
        for (int i = j + lane; i < r; i += 64) w += (i == j ? 1.0 : col[i]) * a[i];
        w = wave_sum(w) * tau;
        for (int i = j + lane; i < r; i += 64) a[i] -= w * (i == j ? 1.0 : col[i]);
      }
    }
    __syncthreads();
    for (int i = tid; i < r; i += kCT) {
      if (i < j) col[i] = 0.0;
      else if (i == j) col[i] = 1.0 - tau;
      else col[i] *= -tau;
    }
    __syncthreads();
  }
  for (int e = tid; e < r * c; e += kCT) {
    const int j = e / r, i = e - j * r;
    T.Q[i + (int64_t)j * T.ldq] = j < nr ? sA[e] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// GEMM tiles: thread (ty, tx) = (tid / 16, tid % 16) owns rows ty + 16 i and
// columns tx + 16 j (i, j < MI) of a 16 MI x 16 MI output (MI = 1..4, picked
// per launch from its largest task, so 36 x 36 blocks take 48 x 48 tiles);
// K in chunks of 32 staged in LDS as sA[k][row], sB[k][col] (odd stride
// against bank conflicts).  Every output sums over k in the same order
// whatever MI.
constexpr int kKc = 32;

template <int MI>
struct GemmAcc {
  double v[MI][MI];
};

__device__ inline double opA(const double* A, int64_t lda, bool t, int i, int k) {
  return t ? A[k + (int64_t)i * lda] : A[i + (int64_t)k * lda];
}

// acc += op(A) (a x K) * op(B) (K x b), operands in global memory
template <int MI>
__device__ void gemm_acc(GemmAcc<MI>& acc, const double* A, int64_t lda, bool ta, const double* B, int64_t ldb,
                         bool tb, int a, int b, int K, double* sA, double* sB) {
  constexpr int TILE = 16 * MI, LD = TILE + 1;
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int k0 = 0; k0 < K; k0 += kKc) {
    const int kc = min(kKc, K - k0);
    __syncthreads();
    for (int e = tid; e < kKc * TILE; e += kCT) {
      // transposed operands: consecutive threads walk k (contiguous), else rows
      int kk, i;
      if (ta) { i = e / kKc; kk = e - i * kKc; } else { kk = e / TILE; i = e - kk * TILE; }
      sA[kk * LD + i] = (kk < kc && i < a) ? opA(A, lda, ta, i, k0 + kk) : 0.0;
    }
    for (int e = tid; e < kKc * TILE; e += kCT) {
      int kk, j;
      if (tb) { kk = e / TILE; j = e - kk * TILE; } else { j = e / kKc; kk = e - j * kKc; }
      // op(B)[k][j] = tb ? B[j][k] : B[k][j]
      sB[kk * LD + j] = (kk < kc && j < b) ? (tb ? B[j + (int64_t)(k0 + kk) * ldb] : B[(k0 + kk) + (int64_t)j * ldb])
                                          : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < kc; ++kk) {
      double ar[MI], br[MI];
#pragma unroll
      for (int i = 0; i < MI; ++i) ar[i] = sA[kk * LD + ty + 16 * i];
#pragma unroll
      for (int j = 0; j < MI; ++j) br[j] = sB[kk * LD + tx + 16 * j];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < MI; ++j) acc.v[i][j] = fma(ar[i], br[j], acc.v[i][j]);
    }
  }
}

template <int MI>
__device__ void gemm_store(const GemmAcc<MI>& acc, double* C, int64_t ldc, int a, int b, double alpha,
                           double beta) {
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MI; ++j) {
      const int row = ty + 16 * i, col = tx + 16 * j;
      if (row < a && col < b) {
        double* o = C + row + (int64_t)col * ldc;
        *o = beta == 0.0 ? alpha * acc.v[i][j] : fma(alpha, acc.v[i][j], beta * *o);
      }
    }
}

template <int MI>
__global__ __launch_bounds__(kCT) void k_gemm(const GemmTask* __restrict__ tasks, const GemmPair* __restrict__ pairs) {
  constexpr int LD = 16 * MI + 1;
  __shared__ double sA[kKc * LD];
  __shared__ double sB[kKc * LD];
  const GemmTask T = tasks[blockIdx.x];
  GemmAcc<MI> acc;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MI; ++j) acc.v[i][j] = 0.0;
  for (int p = T.pbeg; p < T.pend; ++p) {
    const GemmPair P = pairs[p];
    gemm_acc<MI>(acc, P.A, P.lda, P.flags & 1, P.B, P.ldb, P.flags & 2, T.m, T.n, P.k, sA, sB);
  }
  gemm_store<MI>(acc, T.C, T.ldc, T.m, T.n, T.alpha, T.beta);
}

// C = beta C + op(L) M R^T: L M (a x k2) into LDS, then times R^T; the tile
// covers a, b and k2
template <int MI>
__global__ __launch_bounds__(kCT) void k_triple(const TripleTask* __restrict__ tasks) {
  constexpr int TILE = 16 * MI, LD = TILE + 1;
  __shared__ double sA[kKc * LD];
  __shared__ double sB[kKc * LD];
  __shared__ double sT[TILE * LD];  // L M, column-major with stride LD
  const TripleTask T = tasks[blockIdx.x];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  GemmAcc<MI> acc;
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MI; ++j) acc.v[i][j] = 0.0;
  gemm_acc<MI>(acc, T.L, T.ldl, T.flags & 1, T.M, T.ldm, false, T.a, T.k2, T.k1, sA, sB);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MI; ++j) sT[(ty + 16 * i) + (tx + 16 * j) * LD] = acc.v[i][j];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MI; ++j) acc.v[i][j] = 0.0;
  __syncthreads();
  // (L M) from LDS times R^T
  for (int k0 = 0; k0 < T.k2; k0 += kKc) {
    const int kc = min(kKc, T.k2 - k0);
    __syncthreads();
    for (int e = tid; e < kKc * TILE; e += kCT) {
      const int kk = e / TILE, j = e - kk * TILE;
      sB[kk * LD + j] = (kk < kc && j < T.b) ? T.R[j + (int64_t)(k0 + kk) * T.ldr] : 0.0;
    }
    __syncthreads();
    for (int kk = 0; kk < kc; ++kk) {
      double ar[MI], br[MI];
#pragma unroll
      for (int i = 0; i < MI; ++i) ar[i] = sT[(ty + 16 * i) + (k0 + kk) * LD];
#pragma unroll
      for (int j = 0; j < MI; ++j) br[j] = sB[kk * LD + tx + 16 * j];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < MI; ++j) acc.v[i][j] = fma(ar[i], br[j], acc.v[i][j]);
    }
  }
  gemm_store<MI>(acc, T.C, T.ldc, T.a, T.b, 1.0, T.beta);
}

// ---------------------------------------------------------------------------
// Parallel cyclic Jacobi for a symmetric n x n matrix (n <= N), one
// workgroup per matrix, matrix and eigenvectors in LDS (sized by N, so small
// orders leave room for more workgroups per CU): rounds of n'/2 disjoint
// rotations (n' = n rounded up to even; the padding index only meets
// identity rotations), tournament ordering, n' - 1 rounds per sweep, until a
// sweep rotates nothing.  Rotation (c, s) from the 2 x 2 symmetric Schur
// decomposition zeroes A[p][q] in J^T A J, J = [[c, s], [-s, c]].
template <int N>
__global__ __launch_bounds__(kCT) void k_eig(const EigTask* __restrict__ tasks) {
  constexpr int LD = N + 1;
  __shared__ double sA[N * LD];
  __shared__ double sV[N * LD];
  __shared__ double rc[N / 2], rs[N / 2];
  __shared__ int rp[N / 2], rq[N / 2];
  __shared__ int s_rot;
  __shared__ double s_lam[N];
  __shared__ double s_red[kCT];
  const EigTask T = tasks[blockIdx.x];
  const int n = T.n, tid = threadIdx.x;
  const int np = (n + 1) & ~1, half = np / 2;
  double sq = 0.0;
  for (int e = tid; e < n * n; e += kCT) {
    const int j = e / n, i = e - j * n;
    // symmetrize (the inputs are symmetric up to rounding)
    const double a = 0.5 * (T.G[i + (int64_t)j * T.ldg] + T.G[j + (int64_t)i * T.ldg]);
    sA[i * LD + j] = a;
    sV[i * LD + j] = i == j ? 1.0 : 0.0;
    sq += a * a;
  }
  s_red[tid] = sq;
  __syncthreads();
  for (int w = kCT / 2; w > 0; w >>= 1) {
    if (tid < w) s_red[tid] += s_red[tid + w];
    __syncthreads();
  }
  // off-diagonal entries below 1e-16 of the Frobenius norm are not rotated:
  // besides the relative test, this stops the sweeps once only rounding
  // noise among the (many) negligible eigenvalues is left, at an absolute
  // accuracy far below any threshold the truncation applies
  const double floor_abs = 1e-16 * sqrt(s_red[0]);
  for (int sweep = 0; sweep < 40 && np > 1; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      if (tid < half) {
        int p, q;
        if (tid == 0) { p = round; q = np - 1; }
        else { p = (round + tid) % (np - 1); q = (round - tid + (np - 1)) % (np - 1); }
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double app = sA[p * LD + p], aqq = sA[q * LD + q], apq = sA[p * LD + q];
          if (fabs(apq) > 1e-300 && fabs(apq) > floor_abs && fabs(apq) > 1e-15 * sqrt(fabs(app) * fabs(aqq))) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            s_rot = 1;
          }
        }
        rp[tid] = p; rq[tid] = q; rc[tid] = c; rs[tid] = s;
      }
      __syncthreads();
      // rows: p' = c p - s q, q' = s p + c q
      for (int e = tid; e < half * n; e += kCT) {
        const int k = e / n, j = e - k * n;
        const int p = rp[k], q = rq[k];
        if (q < n && rs[k] != 0.0) {
          const double c = rc[k], s = rs[k];
          const double ap = sA[p * LD + j], aq = sA[q * LD + j];
          sA[p * LD + j] = c * ap - s * aq;
          sA[q * LD + j] = s * ap + c * aq;
        }
      }
      __syncthreads();
      // columns of A and V: p'' = c p - s q, q'' = s p + c q
      for (int e = tid; e < half * n; e += kCT) {
        const int k = e / n, i = e - k * n;
        const int p = rp[k], q = rq[k];
        if (q < n && rs[k] != 0.0) {
          const double c = rc[k], s = rs[k];
          const double ap = sA[i * LD + p], aq = sA[i * LD + q];
          sA[i * LD + p] = c * ap - s * aq;
          sA[i * LD + q] = s * ap + c * aq;
          const double vp = sV[i * LD + p], vq = sV[i * LD + q];
          sV[i * LD + p] = c * vp - s * vq;
          sV[i * LD + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
    if (s_rot == 0) break;
    __syncthreads();
  }
  // descending order (ties by index)
  for (int i = tid; i < n; i += kCT) s_lam[i] = sA[i * LD + i];
  __syncthreads();
  for (int i = tid; i < n; i += kCT) {
    const double li = s_lam[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += (s_lam[j] > li) || (s_lam[j] == li && j < i);
    T.lam[rank] = li;
    for (int row = 0; row < n; ++row) T.Z[row + (int64_t)rank * T.ldz] = sV[row * LD + i];
  }
}

// ---------------------------------------------------------------------------
// Elementwise helpers (one workgroup per node)

// masked Gram: out = P G P, P = diag(1 if column j of the leaf basis is nonzero)
__global__ __launch_bounds__(kCT) void k_mask_gram(const MaskTask* __restrict__ tasks) {
  __shared__ int nz[kMaxCompressRank];
  const MaskTask T = tasks[blockIdx.x];
  const int k = T.k, m = T.m, tid = threadIdx.x;
  for (int j = tid; j < k; j += kCT) {
    int any = 0;
    for (int i = 0; i < m; ++i) any |= T.U[i + (int64_t)j * T.ldu] != 0.0;
    nz[j] = any;
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += kCT) {
    const int j = e / k, i = e - j * k;
    T.out[i + (int64_t)j * k] = (nz[i] && nz[j]) ? T.G[i + (int64_t)j * T.ldg] : 0.0;
  }
}

// per node: count of lam > thr2 (first `n` entries), into counts[node]
__global__ void k_count(const CountTask* __restrict__ tasks, int64_t ntasks, double thr2, int32_t* counts) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= ntasks) return;
  const CountTask T = tasks[t];
  int c = 0;
  for (int i = 0; i < T.n; ++i) c += T.lam[i] > thr2;
  counts[T.node] = c;
}

// largest first eigenvalue over the tasks (one workgroup, fixed order)
__global__ __launch_bounds__(kCT) void k_max_lead(const CountTask* __restrict__ tasks, int64_t ntasks,
                                                   double* out) {
  __shared__ double red[kCT];
  double m = 0.0;
  for (int64_t t = threadIdx.x; t < ntasks; t += kCT) {
    const CountTask T = tasks[t];
    if (T.n > 0) m = fmax(m, T.lam[0]);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = kCT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

// column scaling of eigenvector matrices: Z[:, j] *= (j < keep ? f(lam_j) : 0)
// for j < cols, with f = 1 (mode 0) or 1/sqrt(lam) (mode 1); the kept count
// is counts[node]
__global__ __launch_bounds__(kCT) void k_scale_cols(const ScaleTask* __restrict__ tasks, const int32_t* counts,
                                                     int mode) {
  const ScaleTask T = tasks[blockIdx.x];
  const int keep = counts[T.node];
  for (int e = threadIdx.x; e < T.rows * T.cols; e += kCT) {
    const int j = e / T.rows, i = e - j * T.rows;
    double f = 0.0;
    if (j < keep) f = mode == 0 ? 1.0 : 1.0 / sqrt(T.lam[j]);
    T.Z[i + (int64_t)j * T.ldz] *= f;
  }
}

// square-root factor R = diag(sqrt(max(lam, 0))) Z^T (n x n)
__global__ __launch_bounds__(kCT) void k_sqrt_factor(const EigTask* __restrict__ tasks, double* const* outs,
                                                      const int64_t* ldo) {
  const EigTask T = tasks[blockIdx.x];
  double* R = outs[blockIdx.x];
  const int64_t ld = ldo[blockIdx.x];
  for (int e = threadIdx.x; e < T.n * T.n; e += kCT) {
    const int j = e / T.n, i = e - j * T.n;
    R[i + (int64_t)j * ld] = sqrt(fmax(T.lam[i], 0.0)) * T.Z[j + (int64_t)i * T.ldz];
  }
}

// dst (rows x cols, ldd) = src (rows x cols, lds), optionally transposed (dst = src^T)
__global__ __launch_bounds__(kCT) void k_copy(const CopyTask* __restrict__ tasks) {
  const CopyTask T = tasks[blockIdx.x];
  for (int e = threadIdx.x; e < T.rows * T.cols; e += kCT) {
    const int j = e / T.rows, i = e - j * T.rows;
    T.dst[i + (int64_t)j * T.ldd] = T.trans ? T.src[j + (int64_t)i * T.lds] : T.src[i + (int64_t)j * T.lds];
  }
}

inline dim3 grid_of(int64_t n) { return dim3((unsigned)n); }

}  // namespace

hipError_t launch_qr(const QrTask* t, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_qr, grid_of(n), dim3(kCT), 0, s, t);
  return hipGetLastError();
}
hipError_t launch_gemm(const GemmTask* t, int64_t n, const GemmPair* p, hipStream_t s, int maxdim) {
  if (n == 0) return hipSuccess;
  if (maxdim <= 16) hipLaunchKernelGGL((k_gemm<1>), grid_of(n), dim3(kCT), 0, s, t, p);
  else if (maxdim <= 32) hipLaunchKernelGGL((k_gemm<2>), grid_of(n), dim3(kCT), 0, s, t, p);
  else if (maxdim <= 48) hipLaunchKernelGGL((k_gemm<3>), grid_of(n), dim3(kCT), 0, s, t, p);
  else if (maxdim <= kTile) hipLaunchKernelGGL((k_gemm<4>), grid_of(n), dim3(kCT), 0, s, t, p);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_triple(const TripleTask* t, int64_t n, hipStream_t s, int maxdim) {
  if (n == 0) return hipSuccess;
  if (maxdim <= 16) hipLaunchKernelGGL((k_triple<1>), grid_of(n), dim3(kCT), 0, s, t);
  else if (maxdim <= 32) hipLaunchKernelGGL((k_triple<2>), grid_of(n), dim3(kCT), 0, s, t);
  else if (maxdim <= 48) hipLaunchKernelGGL((k_triple<3>), grid_of(n), dim3(kCT), 0, s, t);
  else if (maxdim <= kTile) hipLaunchKernelGGL((k_triple<4>), grid_of(n), dim3(kCT), 0, s, t);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_eig(const EigTask* t, int64_t n, int nmax, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (nmax <= 32) hipLaunchKernelGGL((k_eig<32>), grid_of(n), dim3(kCT), 0, s, t);
  else if (nmax <= 48) hipLaunchKernelGGL((k_eig<48>), grid_of(n), dim3(kCT), 0, s, t);
  else if (nmax <= kMaxCompressRank) hipLaunchKernelGGL((k_eig<64>), grid_of(n), dim3(kCT), 0, s, t);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_mask_gram(const MaskTask* t, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_mask_gram, grid_of(n), dim3(kCT), 0, s, t);
  return hipGetLastError();
}
hipError_t launch_count(const CountTask* t, int64_t n, double thr2, int32_t* counts, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_count, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t, n, thr2, counts);
  return hipGetLastError();
}
hipError_t launch_max_lead(const CountTask* t, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_max_lead, dim3(1), dim3(kCT), 0, s, t, n, out);
  return hipGetLastError();
}
hipError_t launch_scale_cols(const ScaleTask* t, int64_t n, const int32_t* counts, int mode, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_cols, grid_of(n), dim3(kCT), 0, s, t, counts, mode);
  return hipGetLastError();
}
hipError_t launch_sqrt_factor(const EigTask* t, int64_t n, double* const* outs, const int64_t* ldo, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sqrt_factor, grid_of(n), dim3(kCT), 0, s, t, outs, ldo);
  return hipGetLastError();
}
hipError_t launch_copy(const CopyTask* t, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, grid_of(n), dim3(kCT), 0, s, t);
  return hipGetLastError();
}

}  // namespace h2
