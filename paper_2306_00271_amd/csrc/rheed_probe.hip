// Measured FP64 matrix-core throughput, the ceiling the propagation kernels
// are compared against beside the published figure.
#include <hip/hip_runtime.h>

#include "rheed.h"
#include "rheed_internal.h"

namespace rheed {

typedef double pd4 __attribute__((ext_vector_type(4)));

// Every wave runs PEAK_CHAINS independent accumulation chains of
// v_mfma_f64_16x16x4f64 (2048 flop each) with operands held in registers, so
// the matrix pipe never waits on memory or on a dependency.
constexpr int PEAK_CHAINS = 8;

__global__ __launch_bounds__(256) void mfma_f64_peak_kernel(double* out, int iters) {
  const int lane = threadIdx.x & 63;
  const double a = 1.0 + 1.0e-3 * lane, b = 1.0 - 1.0e-3 * lane;
  pd4 c[PEAK_CHAINS];
#pragma unroll
  for (int q = 0; q < PEAK_CHAINS; ++q) c[q] = pd4{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int q = 0; q < PEAK_CHAINS; ++q) c[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[q], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < PEAK_CHAINS; ++q) s += c[q][0] + c[q][1] + c[q][2] + c[q][3];
  out[(long long)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace rheed

using namespace rheed;

extern "C" rheed_status rheed_mfma_f64_peak(int32_t blocks, int32_t iters, double* tflops) {
  if (blocks < 1 || blocks > 65536 || iters < 1 || iters > 1000000 || !tflops) return RHEED_E_INVALID;
  double* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&out, (size_t)blocks * 256 * sizeof(double));
  if (e != hipSuccess) return RHEED_E_NOMEM;
  rheed_status st = RHEED_OK;
  float ms = 0.0f;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = RHEED_E_HIP;
  if (st == RHEED_OK) {
    // one untimed launch, then the timed one
    hipLaunchKernelGGL(mfma_f64_peak_kernel, dim3(blocks), dim3(256), 0, nullptr, out, 1);
    hipEventRecord(e0, nullptr);
    hipLaunchKernelGGL(mfma_f64_peak_kernel, dim3(blocks), dim3(256), 0, nullptr, out, iters);
    hipEventRecord(e1, nullptr);
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.0f)
      st = RHEED_E_HIP;
  }
  if (st == RHEED_OK) {
    const double flop = (double)blocks * 4.0 * (double)iters * PEAK_CHAINS * 2048.0;
    *tflops = flop / (ms * 1.0e-3) / 1.0e12;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(out);
  return st;
}
