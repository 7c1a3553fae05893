// Measured FP64 matrix-core rate of the device: the ceiling the weight build's
// MFMA assembly is compared with, next to the data-sheet peak.
//
// Every wavefront keeps four independent 16x16 accumulators and feeds them
// v_mfma_f64_16x16x4f64 in turn (2048 flops each), so the matrix pipe of
// each SIMD always has independent work; the grid holds eight workgroups of
// four wavefronts per CU.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace labfm {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kChains = 4;

__global__ void __launch_bounds__(256) mfma_f64_rate_kernel(int iters, double* __restrict__ out) {
  double4_t acc[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) acc[k] = double4_t{0.0, 0.0, 0.0, 0.0};
  const double a = 1.0 + 1e-9 * threadIdx.x;
  const double b = 1.0 - 1e-9 * blockIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k)
      acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kChains; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  // every lane writes its own slot: the sums stay live and the stores in bounds
  out[static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

}  // namespace
}  // namespace labfm

using namespace labfm;

extern "C" size_t labfm_mfma_f64_rate_scratch_bytes(void) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return sizeof(double) * static_cast<size_t>(cus) * 8 * 256;
}

extern "C" int labfm_mfma_f64_rate(int32_t iters, double* scratch, size_t scratch_bytes,
                                   double* tflops, void* stream_) {
  clear_error();
  LABFM_REQUIRE(iters > 0 && scratch && tflops, "mfma_f64_rate: bad argument");
  int dev = 0, cus = 0;
  LABFM_HIP(hipGetDevice(&dev));
  LABFM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const unsigned grid = static_cast<unsigned>(cus) * 8;
  LABFM_REQUIRE(scratch_bytes >= sizeof(double) * static_cast<size_t>(grid) * 256,
                "mfma_f64_rate: scratch holds %zu bytes, %zu needed", scratch_bytes,
                sizeof(double) * static_cast<size_t>(grid) * 256);
  hipStream_t st = as_stream(stream_);
  hipEvent_t e0, e1;
  LABFM_HIP(hipEventCreate(&e0));
  LABFM_HIP(hipEventCreate(&e1));
  // one untimed launch, then the timed one
  hipLaunchKernelGGL(mfma_f64_rate_kernel, dim3(grid), dim3(256), 0, st, iters, scratch);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(mfma_f64_rate_kernel, dim3(grid), dim3(256), 0, st, iters, scratch);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  LABFM_HIP(e);
  const double flops = 2048.0 * kChains * static_cast<double>(iters) * grid * 4.0;
  *tflops = ms > 0.0f ? flops / (static_cast<double>(ms) * 1e-3) / 1e12 : 0.0;
  return LABFM_OK;
}
