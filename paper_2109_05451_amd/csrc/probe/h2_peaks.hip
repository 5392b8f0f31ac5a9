// Measured peaks of the GPU the benchmark runs on, reported beside the
// datasheet figures: the HBM read rate of a streaming kernel (16-byte
// nontemporal loads, grid-stride) and the FP64 and BF16 matrix-core rates of
// a loop of independent MFMA chains.  Benchmark support only; the product
// library does not use this.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(256) void k_read(const d2* __restrict__ src, int64_t n2, double* __restrict__ sink) {
  d2 acc = {0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
    acc += __builtin_nontemporal_load(src + i);
  if (acc.x == 1234.5 && acc.y == -1.0) sink[0] = acc.x;  // keeps the loads live
}

// Four independent accumulator chains per wave, ITERS steps each.
__global__ __launch_bounds__(256) void k_mfma_f64(int iters, double seed, double* __restrict__ sink) {
  d4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  const double a = seed + threadIdx.x * 1e-9, b = seed - threadIdx.x * 1e-9;
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c3, 0, 0, 0);
  }
  const double r = c0[0] + c1[1] + c2[2] + c3[3];
  if (r == 1234.5) sink[0] = r;
}

__global__ __launch_bounds__(256) void k_mfma_bf16(int iters, float seed, double* __restrict__ sink) {
  f4 c0 = {0, 0, 0, 0}, c1 = c0, c2 = c0, c3 = c0;
  bf8 a, b;
  for (int k = 0; k < 8; ++k) {
    a[k] = (__bf16)(seed + k + threadIdx.x * 1e-3f);
    b[k] = (__bf16)(seed - k);
  }
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c3, 0, 0, 0);
  }
  const float r = c0[0] + c1[1] + c2[2] + c3[3];
  if (r == 1234.5f) sink[0] = r;
}

template <class F>
int timed(F launch, int reps, float* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = -1;
  if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
    launch();  // warm-up
    if (hipEventRecord(e0, nullptr) == hipSuccess) {
      for (int r = 0; r < reps; ++r) launch();
      if (hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
          hipEventElapsedTime(ms, e0, e1) == hipSuccess && hipGetLastError() == hipSuccess) {
        *ms /= reps;
        rc = 0;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return rc;
}

}  // namespace

extern "C" {

// Average time (ms) of one read of `bytes` (a multiple of 16) of device memory at `buf`.
int h2p_read(const void* buf, int64_t bytes, void* sink, int reps, float* ms) {
  int ncu = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  const unsigned grid = (unsigned)(ncu * 8);
  return timed([&] { hipLaunchKernelGGL(k_read, dim3(grid), dim3(256), 0, nullptr, static_cast<const d2*>(buf),
                                        bytes / 16, static_cast<double*>(sink)); },
               reps, ms);
}

// Average time (ms) of a launch of `waves_per_simd` waves on every SIMD,
// each `iters` x 4 MFMAs; *flops receives the flops of one launch.
int h2p_mfma(int bf16, int iters, int waves_per_simd, void* sink, float* ms, double* flops) {
  int ncu = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  const unsigned grid = (unsigned)(ncu * waves_per_simd);  // 4 waves (one per SIMD) per workgroup
  const double per = bf16 ? 16.0 * 16 * 32 * 2 : 16.0 * 16 * 4 * 2;
  *flops = (double)grid * 4 * iters * 4 * per;
  if (bf16)
    return timed([&] { hipLaunchKernelGGL(k_mfma_bf16, dim3(grid), dim3(256), 0, nullptr, iters, 1.0f,
                                          static_cast<double*>(sink)); },
                 3, ms);
  return timed([&] { hipLaunchKernelGGL(k_mfma_f64, dim3(grid), dim3(256), 0, nullptr, iters, 1.0,
                                        static_cast<double*>(sink)); },
               3, ms);
}

}  // extern "C"
