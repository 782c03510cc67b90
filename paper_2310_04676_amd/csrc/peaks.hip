// Measured peaks of the device, the denominators a roofline fraction can be
// quoted against besides the datasheet ones: FP32 VALU FMA issue (with the
// packed-FP32 instructions the library is compiled without, as every kernel sees
// it) for a full chip and for a wave alone on its SIMD, BF16 matrix-core
// issue (v_mfma_f32_16x16x32_bf16), and a streaming device-to-device copy.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "mlp.hpp"

namespace sgk {

constexpr int kPeakChains = 16;

// Independent FMA chains per lane; the result is stored (if a sentinel
// value is hit) so the loop cannot be removed.
__global__ void __launch_bounds__(256) k_peak_fma(int iters, float seed, float* sink) {
  float a[kPeakChains];
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) a[c] = seed + 0.001f * (threadIdx.x + c);
  const float m = 0.9999f, b = 1e-6f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) a[c] = fmaf(a[c], m, b);
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kPeakChains; ++c) s += a[c];
  if (s == 12345.678f) sink[blockIdx.x] = s;
}

// Eight independent accumulators of 16x16x32 BF16 MFMAs per wave.
__global__ void __launch_bounds__(256) k_peak_mfma(int iters, float* sink) {
  bf16x8 a, b;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    a[s] = (__bf16)(0.01f * (threadIdx.x + s));
    b[s] = (__bf16)(0.02f * (threadIdx.x - s));
  }
  f32x4 c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = mfma16x16x32((k & 1) ? a : b, (k & 2) ? a : b, c[k]);
  }
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += c[k][k & 3];
  if (s == 12345.678f) sink[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_peak_copy(const float4* __restrict__ src, float4* __restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) dst[i] = src[i];
}

}  // namespace sgk

extern "C" sg_status sg_measure_peaks(double* fp32_fma_tflops, double* fp32_fma_wave_gflops, double* bf16_mfma_tflops,
                                      double* copy_gbps) {
  if (!fp32_fma_tflops || !fp32_fma_wave_gflops || !bf16_mfma_tflops || !copy_gbps) return SG_E_INVAL;
  int dev = 0, n_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t copy_bytes = (size_t)1 << 30;
  float* sink = nullptr;
  void *src = nullptr, *dst = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipMalloc((void**)&sink, 65536 * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&src, copy_bytes);
  if (e == hipSuccess) e = hipMalloc(&dst, copy_bytes);
  if (e == hipSuccess) e = hipMemset(src, 0, copy_bytes);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  // eight 256-thread blocks per CU: two waves per SIMD
  const int blocks = 8 * (n_cu > 0 ? n_cu : 256);
  float ms = 0.f;
  // average milliseconds per launch; a HIP error is kept in e
  auto timed = [&](auto launch, int reps) -> float {
    launch();  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, nullptr);
    for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
    if (e == hipSuccess) e = hipEventRecord(e1, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    return e == hipSuccess && t > 0.f ? t / reps : 1.f;
  };
  if (e == hipSuccess) {
    const int iters = 4096;
    ms = timed([&] { sgk::k_peak_fma<<<blocks, 256>>>(iters, 1.f, sink); }, 5);
    *fp32_fma_tflops = 2.0 * sgk::kPeakChains * (double)iters * blocks * 256 / (ms * 1e-3) / 1e12;
    // one single-wave workgroup per CU: each wave alone on its SIMD
    const int lone = n_cu > 0 ? n_cu : 256;
    ms = timed([&] { sgk::k_peak_fma<<<lone, 64>>>(iters, 1.f, sink); }, 5);
    *fp32_fma_wave_gflops = 2.0 * sgk::kPeakChains * (double)iters * 64 / (ms * 1e-3) / 1e9;
    // sixteen 256-thread blocks per CU: four waves per SIMD
    const int mi = 1024, mblocks = 2 * blocks;
    ms = timed([&] { sgk::k_peak_mfma<<<mblocks, 256>>>(mi, sink); }, 5);
    *bf16_mfma_tflops = 8.0 * mi * 2.0 * 16 * 16 * 32 * (double)mblocks * 4 / (ms * 1e-3) / 1e12;
    const size_t n4 = copy_bytes / 16;
    ms = timed([&] { sgk::k_peak_copy<<<blocks, 256>>>((const float4*)src, (float4*)dst, n4); }, 5);
    *copy_gbps = 2.0 * copy_bytes / (ms * 1e-3) / 1e9;
    if (e == hipSuccess) e = hipGetLastError();
  }
  void* ptrs[] = {sink, src, dst};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e == hipSuccess ? SG_OK : SG_E_HIP;
}
