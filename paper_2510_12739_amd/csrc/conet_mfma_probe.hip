// One matrix instruction of the kinds the conv kernels use, on caller-given operands: how the
// instruction accumulates its products (which the parity tolerances model) can be checked on
// any device. Every row of A holds a[0..K) and every column of B holds b[0..K), so every
// output element is the instruction's sum of a[k] b[k].
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "conet.h"
#include "conet_common.h"
#include "conet_model.h"

namespace conet {

// SHAPE 16: 16x16xK, lane l supplies row / column l % 16 and K block l / 16 (K/4 values);
// SHAPE 32: 32x32xK, lane l supplies row / column l % 32 and K block l / 32 (K/2 values).
template <int DT, int SHAPE>
__global__ void __launch_bounds__(64) mfma_dot_kernel(const uint8_t* __restrict__ a, const uint8_t* __restrict__ b,
                                                      float* __restrict__ out) {
  const int l = threadIdx.x;
  if constexpr (DT == DT_BF16) {
    constexpr int KB = SHAPE == 16 ? 8 : 8;  // 8 BF16 values per lane in both shapes
    const int kb = SHAPE == 16 ? l / 16 : l / 32;
    bf16x8 av, bv;
    memcpy(&av, a + kb * KB * 2, 16);
    memcpy(&bv, b + kb * KB * 2, 16);
    if constexpr (SHAPE == 16) {
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
      if (l == 0) out[0] = c[0];
    } else {
      f32x16 c = {};
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
      if (l == 0) out[0] = c[0];
    }
  } else {
    const int kb = SHAPE == 16 ? l / 16 : l / 32;  // 32 e4m3 values per lane in both shapes
    i32x8 av, bv;
    memcpy(&av, a + kb * 32, 32);
    memcpy(&bv, b + kb * 32, 32);
    if constexpr (SHAPE == 16) {
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
      c = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, c, 0, 0, 0, 0, 0, 0);
      if (l == 0) out[0] = c[0];
    } else {
      f32x16 c = {};
      c = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av, bv, c, 0, 0, 0, 0, 0, 0);
      if (l == 0) out[0] = c[0];
    }
  }
}

}  // namespace conet

using namespace conet;

extern "C" conet_status conet_mfma_dot(int32_t dtype, int32_t shape, const void* a_host, const void* b_host,
                                       float* out_host) {
  if (!a_host || !b_host || !out_host) return fail(CONET_EINVAL, "null argument");
  if (shape != 16 && shape != 32) return fail(CONET_EINVAL, "shape must be 16 or 32");
  int K = 0, esize = 0;
  if (dtype == DT_BF16) { K = shape == 16 ? 32 : 16; esize = 2; }
  else if (dtype == DT_FP8) { K = shape == 16 ? 128 : 64; esize = 1; }
  else return fail(CONET_EINVAL, "dtype must be BF16 or FP8");
  const size_t bytes = (size_t)K * esize;
  uint8_t* dev = nullptr;
  hipError_t e = hipMalloc(&dev, 2 * bytes + 16);
  if (e != hipSuccess) return hip_fail(e, "probe buffer");
  float* dout = reinterpret_cast<float*>(dev + 2 * bytes);
  e = hipMemcpy(dev, a_host, bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dev + bytes, b_host, bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    const dim3 g(1), blk(64);
    if (dtype == DT_BF16 && shape == 16) hipLaunchKernelGGL((mfma_dot_kernel<DT_BF16, 16>), g, blk, 0, 0, dev, dev + bytes, dout);
    else if (dtype == DT_BF16) hipLaunchKernelGGL((mfma_dot_kernel<DT_BF16, 32>), g, blk, 0, 0, dev, dev + bytes, dout);
    else if (shape == 16) hipLaunchKernelGGL((mfma_dot_kernel<DT_FP8, 16>), g, blk, 0, 0, dev, dev + bytes, dout);
    else hipLaunchKernelGGL((mfma_dot_kernel<DT_FP8, 32>), g, blk, 0, 0, dev, dev + bytes, dout);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(out_host, dout, sizeof(float), hipMemcpyDeviceToHost);
  const hipError_t ef = hipFree(dev);
  if (e == hipSuccess) e = ef;
  if (e != hipSuccess) return hip_fail(e, "MFMA probe");
  return CONET_OK;
}
