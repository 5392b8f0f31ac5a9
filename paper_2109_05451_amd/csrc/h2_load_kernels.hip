// Kernels run once when an operator is loaded.
#include <algorithm>

#include "h2_internal.h"

namespace h2 {
namespace {

// The transposed copies of the leaf bases and transfer matrices (used by the
// upsweep products): task b's column-major rows x cols block at mat + src
// becomes its transpose (cols x rows, column-major) at trans + dst.  One
// workgroup per task, grid-stride; reads are contiguous.
__global__ __launch_bounds__(256) void k_transpose_tasks(const TransTask* __restrict__ tasks, int64_t ntasks,
                                                          const double* __restrict__ mat,
                                                          double* __restrict__ trans) {
  for (int64_t b = blockIdx.x; b < ntasks; b += gridDim.x) {
    const TransTask T = tasks[b];
    const int64_t total = (int64_t)T.rows * T.cols;
    for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
      const int64_t r = e % T.rows, c = e / T.rows;
      trans[T.dst + c + (int64_t)T.cols * r] = mat[T.src + e];
    }
  }
}

}  // namespace

hipError_t launch_transpose_tasks(const TransTask* tasks, int64_t ntasks, const double* mat, double* trans,
                                  hipStream_t s) {
  if (ntasks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_transpose_tasks, dim3((unsigned)std::min<int64_t>(ntasks, 65536)), dim3(256), 0, s, tasks,
                     ntasks, mat, trans);
  return hipGetLastError();
}

}  // namespace h2
