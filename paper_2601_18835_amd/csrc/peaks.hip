// Ceilings of the GPU this library runs on, measured by its own
// microbenchmarks (the datasheet peaks are what rooflines are priced
// against; these show what this code generation reaches):
//   FP32 and FP64 FMA issue: independent dependent-chain fused multiply-adds,
//     compiled like every kernel here (packed FP32 off);
//   BF16 MFMA: independent chains of 16x16x32 products with FP32 accumulation
//     (the instruction of the hi/lo FIR);
//   HBM: a device-to-device copy of 1 GiB, read + write bytes over time.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "rfd_internal.h"

namespace rfd {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8_p;
typedef __attribute__((ext_vector_type(4))) float f32x4_p;

constexpr int kPeakIters = 4096;
constexpr int kPeakChains = 16;

template <typename T>
__global__ __launch_bounds__(256) void k_peak_fma(T* __restrict__ out, T b, T c) {
  T a[kPeakChains];
#pragma unroll
  for (int i = 0; i < kPeakChains; ++i) a[i] = (T)threadIdx.x * (T)1e-3 + (T)i;
  for (int it = 0; it < kPeakIters; ++it) {
#pragma unroll
    for (int i = 0; i < kPeakChains; ++i) a[i] = a[i] * b + c;
  }
  T s = 0;
#pragma unroll
  for (int i = 0; i < kPeakChains; ++i) s += a[i];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_mfma(float* __restrict__ out) {
  constexpr int kAcc = 4;
  bf16x8_p a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(1e-3f * (threadIdx.x + i));
    b[i] = (__bf16)(1e-3f * i);
  }
  f32x4_p acc[kAcc];
#pragma unroll
  for (int k = 0; k < kAcc; ++k) acc[k] = f32x4_p{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < kPeakIters / 4; ++it) {
#pragma unroll
    for (int k = 0; k < kAcc; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < kAcc; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_copy(const float4* __restrict__ src, float4* __restrict__ dst,
                                                 int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

}  // namespace rfd

using namespace rfd;

extern "C" {

int rfd_measure_peaks(void* stream, double* out) {
  if (!out) return fail(RFD_E_INVALID, "out is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  int dev = 0, ncu = 0;
  RFD_HIP(hipGetDevice(&dev));
  RFD_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int blocks = std::max(ncu, 1) * 32;
  const size_t copy_bytes = (size_t)1 << 30;
  void* res = nullptr;
  void* a = nullptr;
  void* b = nullptr;
  if (device_malloc((void**)&res, (size_t)blocks * 256 * sizeof(double)) != hipSuccess ||
      device_malloc((void**)&a, copy_bytes) != hipSuccess || device_malloc((void**)&b, copy_bytes) != hipSuccess) {
    (void)hipGetLastError();
    if (res) (void)hipFree(res);
    if (a) (void)hipFree(a);
    return fail(RFD_E_NOMEM, "peaks: hipMalloc failed");
  }
  hipEvent_t e0, e1;
  int rc = RFD_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(RFD_E_DEVICE, "event");
  // best of three launches each (the first also warms the code)
  auto best = [&](auto launch) -> double {
    double ms_best = 1e30;
    for (int r = 0; r < 3 && !rc; ++r) {
      (void)hipEventRecord(e0, st);
      launch();
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess || hipGetLastError() != hipSuccess) {
        rc = fail(RFD_E_DEVICE, "peak kernel failed");
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms_best = std::min<double>(ms_best, ms);
    }
    return ms_best;
  };
  const double lanes = (double)blocks * 256;
  double ms = best([&] {
    hipLaunchKernelGGL(k_peak_fma<float>, dim3(blocks), dim3(256), 0, st, (float*)res, 0.999f, 1e-3f);
  });
  out[0] = lanes * kPeakIters * kPeakChains * 2.0 / (ms * 1e-3) / 1e12;
  ms = best([&] {
    hipLaunchKernelGGL(k_peak_fma<double>, dim3(blocks), dim3(256), 0, st, (double*)res, 0.999, 1e-3);
  });
  out[1] = lanes * kPeakIters * kPeakChains * 2.0 / (ms * 1e-3) / 1e12;
  ms = best([&] { hipLaunchKernelGGL(k_peak_mfma, dim3(blocks), dim3(256), 0, st, (float*)res); });
  // per wave: kPeakIters / 4 iterations x 4 products of 2 x 16 x 16 x 32 flop
  out[2] = (double)blocks * 4 * (kPeakIters / 4) * 4 * (2.0 * 16 * 16 * 32) / (ms * 1e-3) / 1e12;
  const int64_t n4 = (int64_t)(copy_bytes / sizeof(float4));
  ms = best([&] {
    hipLaunchKernelGGL(k_peak_copy, dim3(blocks * 4), dim3(256), 0, st, (const float4*)a, (float4*)b, n4);
  });
  out[3] = 2.0 * (double)copy_bytes / (ms * 1e-3) / 1e9;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(res);
  (void)hipFree(a);
  (void)hipFree(b);
  return rc;
}

}  // extern "C"
