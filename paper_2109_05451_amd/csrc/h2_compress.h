// Internal declarations of the recompression path (Section 5 of the paper):
// task descriptors of its batched kernels and their launchers.  Every task
// describes column-major matrices by pointer, leading dimension and sizes;
// the host builds and bounds-checks them, one workgroup runs each.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace h2 {

constexpr int kMaxCompressRank = 64;    // ranks (and eigenproblem orders) handled
constexpr int kQrMaxElems = 8192;       // rows * cols of one QR operand (64 KiB of LDS)

struct QrTask {  // A = Q R; Q (rows x cols) may alias A; R (cols x cols)
  const double* A;
  int64_t lda;
  double* Q;
  int64_t ldq;
  double* R;
  int64_t ldr;
  int32_t rows, cols;
};

struct GemmTask {  // C (m x n) = beta C + alpha sum over pairs [pbeg, pend)
  double* C;
  int64_t ldc;
  double alpha, beta;
  int32_t m, n;
  int32_t pbeg, pend;
};

struct GemmPair {  // op(A) (m x k) op(B) (k x n); flags bit0: A^T, bit1: B^T
  const double* A;
  const double* B;
  int64_t lda, ldb;
  int32_t k;
  int32_t flags;
};

struct TripleTask {  // C (a x b) = beta C + op(L) (a x k1) M (k1 x k2) R^T (R: b x k2)
  const double* L;
  const double* M;
  const double* R;
  double* C;
  int64_t ldl, ldm, ldr, ldc;
  int32_t a, k1, k2, b;
  double beta;
  int32_t flags;  // bit0: L is stored transposed (k1 x a)
  int32_t pad;
};

struct EigTask {  // G (n x n, symmetric) = Z diag(lam) Z^T, lam descending
  const double* G;
  int64_t ldg;
  double* lam;
  double* Z;
  int64_t ldz;
  int32_t n;
  int32_t pad;
};

struct MaskTask {  // out (k x k) = P G P, P_jj = 1 iff column j of U (m x k) is nonzero
  const double* U;
  int64_t ldu;
  const double* G;
  int64_t ldg;
  double* out;
  int32_t m, k;
};

struct CountTask {  // counts[node] = #{i < n : lam[i] > threshold}
  const double* lam;
  int32_t n;
  int32_t node;
};

struct ScaleTask {  // Z[:, j] *= (j < counts[node] ? f(lam[j]) : 0), j < cols
  double* Z;
  int64_t ldz;
  const double* lam;
  int32_t rows, cols;
  int32_t node;
  int32_t pad;
};

struct CopyTask {  // dst (rows x cols) = trans ? src^T : src
  const double* src;
  double* dst;
  int64_t lds, ldd;
  int32_t rows, cols;
  int32_t trans;
  int32_t pad;
};

hipError_t launch_qr(const QrTask* t, int64_t n, hipStream_t s);
// maxdim: the largest output dimension over the tasks (and, for the triple
// product, the inner dimension k2); it picks the tile, at most 64
hipError_t launch_gemm(const GemmTask* t, int64_t n, const GemmPair* p, hipStream_t s, int maxdim);
hipError_t launch_triple(const TripleTask* t, int64_t n, hipStream_t s, int maxdim);
hipError_t launch_eig(const EigTask* t, int64_t n, int nmax, hipStream_t s);  // nmax: largest order
hipError_t launch_mask_gram(const MaskTask* t, int64_t n, hipStream_t s);
hipError_t launch_count(const CountTask* t, int64_t n, double thr2, int32_t* counts, hipStream_t s);
hipError_t launch_max_lead(const CountTask* t, int64_t n, double* out, hipStream_t s);
hipError_t launch_scale_cols(const ScaleTask* t, int64_t n, const int32_t* counts, int mode, hipStream_t s);
hipError_t launch_sqrt_factor(const EigTask* t, int64_t n, double* const* outs, const int64_t* ldo, hipStream_t s);
hipError_t launch_copy(const CopyTask* t, int64_t n, hipStream_t s);

}  // namespace h2
