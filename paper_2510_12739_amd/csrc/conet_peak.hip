// Dense-MFMA throughput microbenchmark: the attainable peak that the forward kernels'
// roofline fractions can be read against (the datasheet figure assumes the peak engine
// clock; a long MFMA-bound run settles at a lower one).
//
// Every wave keeps NACC independent 16x16 accumulators and issues them round-robin, so
// the matrix pipe never waits on a dependency; operands stay in registers. Wave 0 of
// work-group 0 also samples the shader clock against the constant-rate real-time
// counter over its loop, which gives the effective clock under full load.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "conet.h"
#include "conet_common.h"
#include "conet_model.h"

namespace conet {

constexpr int PEAK_NACC = 8;

// Eight named accumulators: with an array the register allocator rotates the
// accumulators through the AGPR file, and the fix-up moves wait on the last MFMA.
#define CONET_PEAK_ROUND(OP) \
  c0 = OP(c0); c1 = OP(c1); c2 = OP(c2); c3 = OP(c3); c4 = OP(c4); c5 = OP(c5); c6 = OP(c6); c7 = OP(c7);

template <int DT>
__global__ void __launch_bounds__(256) mfma_peak_kernel(int iters, float* __restrict__ sink,
                                                        unsigned long long* __restrict__ clk) {
  const int lane = threadIdx.x & 63;
  const float z = (float)lane;
  f32x4 c0 = {z, z, z, z}, c1 = c0 + 1.f, c2 = c0 + 2.f, c3 = c0 + 3.f, c4 = c0 + 4.f, c5 = c0 + 5.f, c6 = c0 + 6.f,
        c7 = c0 + 7.f;
  const unsigned long long t0 = clock64(), w0 = wall_clock64();
  if constexpr (DT == DT_BF16) {
    bf16x8 a, b;
#pragma unroll
    for (int s = 0; s < 8; ++s) { a[s] = (__bf16)(0.001f * (lane + s)); b[s] = (__bf16)(0.002f * (lane - s)); }
    auto op = [&](f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); };
    for (int it = 0; it < iters; ++it) { CONET_PEAK_ROUND(op) }
  } else if constexpr (DT == DT_FP8) {
    i32x8 a, b;
#pragma unroll
    for (int s = 0; s < 8; ++s) { a[s] = 0x38383838 + lane; b[s] = 0x30303030 + s; }
    auto op = [&](f32x4 c) { return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0); };
    for (int it = 0; it < iters; ++it) { CONET_PEAK_ROUND(op) }
  } else {
    const float a = 0.001f * lane, b = 0.002f * lane;
    auto op = [&](f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); };
    for (int it = 0; it < iters; ++it) { CONET_PEAK_ROUND(op) }
  }
  const unsigned long long t1 = clock64(), w1 = wall_clock64();
  const f32x4 sum = c0 + c1 + c2 + c3 + c4 + c5 + c6 + c7;
  sink[blockIdx.x * blockDim.x + threadIdx.x] = sum[0] + sum[1] + sum[2] + sum[3];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    clk[0] = t1 - t0;
    clk[1] = w1 - w0;
  }
}
#undef CONET_PEAK_ROUND

}  // namespace conet

using namespace conet;

extern "C" conet_status conet_mfma_peak(int32_t dtype, int32_t iters, double* tflops_host, double* clock_ghz_host,
                                        void* stream) {
  if (!tflops_host || !clock_ghz_host) return fail(CONET_EINVAL, "null output");
  if (dtype != DT_F32 && dtype != DT_BF16 && dtype != DT_FP8) return fail(CONET_EINVAL, "dtype must be FP32, BF16 or FP8");
  if (iters < 1 || iters > (1 << 24)) return fail(CONET_EINVAL, "iters must be 1..2^24");
  hipStream_t s = (hipStream_t)stream;
  int dev = 0, n_cu = 0, wall_khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess) return hip_fail(e, "device query");
  const int blocks = n_cu * 4;  // 16 waves per CU: 4 per SIMD
  float* sink = nullptr;
  unsigned long long* clk = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  e = hipMalloc(&sink, (size_t)blocks * 256 * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&clk, 2 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float ms = 0.f;
  unsigned long long clk_h[2] = {0, 0};
  auto launch = [&]() -> hipError_t {
    if (dtype == DT_BF16)
      hipLaunchKernelGGL(mfma_peak_kernel<DT_BF16>, dim3(blocks), dim3(256), 0, s, iters, sink, clk);
    else if (dtype == DT_FP8)
      hipLaunchKernelGGL(mfma_peak_kernel<DT_FP8>, dim3(blocks), dim3(256), 0, s, iters, sink, clk);
    else
      hipLaunchKernelGGL(mfma_peak_kernel<DT_F32>, dim3(blocks), dim3(256), 0, s, iters, sink, clk);
    return hipGetLastError();
  };
  if (e == hipSuccess) e = launch();  // warm-up (clock ramp)
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) e = hipMemcpy(clk_h, clk, sizeof(clk_h), hipMemcpyDeviceToHost);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (sink) (void)hipFree(sink);
  if (clk) (void)hipFree(clk);
  if (e != hipSuccess) return hip_fail(e, "MFMA peak run");
  const double flop_per_mfma = dtype == DT_BF16 ? 2.0 * 16 * 16 * 32 : dtype == DT_FP8 ? 2.0 * 16 * 16 * 128 : 2.0 * 16 * 16 * 4;
  const double waves = (double)blocks * 4;
  *tflops_host = waves * iters * PEAK_NACC * flop_per_mfma / (ms * 1e-3) / 1e12;
  // shader cycles / real-time ticks x real-time rate
  *clock_ghz_host = (clk_h[1] && wall_khz > 0) ? (double)clk_h[0] / (double)clk_h[1] * wall_khz * 1e-6 : 0.0;
  return CONET_OK;
}
