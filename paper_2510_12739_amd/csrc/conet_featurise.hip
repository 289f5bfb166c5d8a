// Input featuriser of CoNet-Rx on the GPU: least-squares channel estimation at the
// pilots, linear interpolation over the resource grid, and the network's input layout.
//
// The receiver's input is the received grid of one TTI (Sec. II, Eq. (1)); the network
// reads, per RE and antenna, the received sample and a channel estimate (Sec. II-A:
// real and imaginary parts as separate channels). Pilots are fixed: symbols 2 and 11,
// even subcarriers, value p = (1 + j)/sqrt(2). Per antenna:
//   * on each pilot symbol s, H_s(f) = y(s, f) / p on even f; an odd f takes the mean of
//     its two even neighbours, and a last odd subcarrier copies its left neighbour;
//   * every symbol t lies on the line through symbols 2 and 11:
//     H(t, f) = H_2(f) + (t - 2) / 9 * (H_11(f) - H_2(f)).
// The known noise and interference variances of each slot can be appended (Sec. II-A
// concatenates them with the received grid). One thread per (slot, subcarrier, antenna)
// forms the two pilot-symbol estimates once and walks the slot's symbols, writing the
// antenna's four channels (Re y, Im y, Re H, Im H) as one 16-byte store per RE;
// neighbouring threads cover neighbouring subcarriers, so every symbol's loads and stores
// are contiguous. Memory-bound: 8 B read and 16 B written per RE and antenna.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "conet.h"
#include "conet_model.h"

namespace conet {

// n_groups = C_in / 4 float4 groups per RE: groups n < n_ant_out are antenna n's (zeros for
// n >= n_rx); with `var` ([B] pairs sigma_n^2, sigma_i^2), the last two groups hold the slot's
// variances and zeros.
__global__ void __launch_bounds__(256) featurise_kernel(const float2* __restrict__ y, const float2* __restrict__ var,
                                                        int64_t n_items, int T, int F, int n_rx, int n_ant_out,
                                                        int n_groups, float4* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  // item = (b * F + f) * n_groups + n; the thread walks the slot's T symbols
  const int n = (int)(i % n_groups);
  const int64_t bf = i / n_groups;
  const int f = (int)(bf % F);
  const int64_t b = bf / F;
  const int64_t slot0 = b * T * F;  // RE index of (b, 0, 0)
  const int64_t sym = (int64_t)F * n_groups;  // stride of one symbol in groups
  float4* xp = x + (slot0 + f) * n_groups + n;
  if (n >= n_ant_out) {  // the variance groups
    const float2 v = var[b];
    const float4 w = n == n_ant_out ? make_float4(v.x, v.y, 0.f, 0.f) : make_float4(0.f, 0.f, 0.f, 0.f);
    for (int t = 0; t < T; ++t) xp[t * sym] = w;
    return;
  }
  if (n >= n_rx) {  // antennas the model has but the grid does not: zero channels
    for (int t = 0; t < T; ++t) xp[t * sym] = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  const float2 h0 = pilot_row_estimate(y + (slot0 + (int64_t)PILOT_T0 * F) * n_rx + n, n_rx, f, F);
  const float2 h1 = pilot_row_estimate(y + (slot0 + (int64_t)PILOT_T1 * F) * n_rx + n, n_rx, f, F);
  const float2* yp = y + (slot0 + f) * n_rx + n;
  for (int t = 0; t < T; ++t) {
    const float2 yv = yp[(int64_t)t * F * n_rx];
    const float2 h = interp_symbol(h0, h1, t);
    xp[(int64_t)t * sym] = make_float4(yv.x, yv.y, h.x, h.y);
  }
}

}  // namespace conet

using namespace conet;

static conet_status featurise(const float* y, const float* var, int32_t B, int32_t T, int32_t F, int32_t n_rx,
                              int32_t C_in, float* x_out, void* stream) {
  if (!y || !x_out) return fail(CONET_EINVAL, "null buffer");
  if (B < 1 || F < 1 || T <= PILOT_T1 || T > TMAX) return fail(CONET_ESHAPE, "need B >= 1, F >= 1, 12 <= T <= 14");
  const int extra = var ? 8 : 0;
  if (n_rx < 1 || C_in < 4 + extra || C_in % 4 != 0 || 4 * n_rx > C_in - extra)
    return fail(CONET_ESHAPE, "need 1 <= n_rx and 4 * n_rx <= C_in%s, C_in a multiple of 4", var ? " - 8" : "");
  const int n_groups = C_in / 4, n_ant_out = (C_in - extra) / 4;
  const int64_t n_items = (int64_t)B * F * n_groups;  // one thread per (slot, subcarrier, group)
  const int64_t blocks = (n_items + 255) / 256;
  if (blocks > 0x7fffffff) return fail(CONET_ESHAPE, "grid too large");
  hipLaunchKernelGGL(featurise_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     reinterpret_cast<const float2*>(y), reinterpret_cast<const float2*>(var), n_items, (int)T,
                     (int)F, (int)n_rx, n_ant_out, n_groups, reinterpret_cast<float4*>(x_out));
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "featurise launch");
  return CONET_OK;
}

extern "C" conet_status conet_featurise(const float* y, int32_t B, int32_t T, int32_t F, int32_t n_rx, int32_t C_in,
                                        float* x_out, void* stream) {
  return featurise(y, nullptr, B, T, F, n_rx, C_in, x_out, stream);
}

extern "C" conet_status conet_featurise_var(const float* y, const float* variances, int32_t B, int32_t T, int32_t F,
                                            int32_t n_rx, int32_t C_in, float* x_out, void* stream) {
  if (!variances) return fail(CONET_EINVAL, "null variances");
  return featurise(y, variances, B, T, F, n_rx, C_in, x_out, stream);
}
