// On-device OFDM slot generator for training batches (the step before the receiver's input,
// Sec. II, Eq. (1)): random bits, Gray QAM with the fixed pilots, a Rayleigh TDL channel whose
// taps vary in time by Clarke's isotropic scattering (a sum of 16 sinusoids per tap and
// antenna), and white Gaussian noise at a random SNR -- so training never waits for the host.
//
// Every random number comes from Philox4x32-10 (Salmon et al., SC 2011) keyed by the seed and
// counted by (slot, stream, index, 0), so a slot is the same whichever batch generates it, and
// the host reference generator (same definition) reproduces it: bits exactly, samples to
// FP32 rounding. Streams: 1 slot parameters, 2 bits, 3 noise, 4 sinusoid angles and phases.
//
// One work-group per (slot, OFDM symbol): its first threads form the channel taps of that
// symbol, g_{l,n}(t) = M^-1/2 sum_s exp(j (2 pi f_D T_sym t cos a_s + p_s)), into LDS; then
// each thread walks subcarriers: bits -> QAM (pilot on pilot REs), H_n = sum_l sqrt(p_l)
// g_{l,n} exp(-j 2 pi f df tau_l), y_n = H_n x + noise_n. Writes y as FP32 [RE][n_rx][2]
// (the featuriser's layout), bits as uint8 [RE][m], and the noise variance of every slot.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "conet.h"
#include "conet_model.h"

namespace conet {

constexpr int SIM_PATHS = 16;
constexpr int SIM_LMAX = 16, SIM_NMAX = 8;
constexpr double SIM_SYMBOL_PERIOD_S = 0.5e-3 / 14.0;  // 14 symbols per 0.5 ms slot (30 kHz numerology)
constexpr double SIM_SUBCARRIER_HZ = 30e3;
constexpr double SIM_TAP_SPACING_S = 200e-9;
constexpr double SIM_PDP_DECAY_S = 300e-9;

struct Philox {
  uint32_t k0, k1;
  __device__ __forceinline__ uint4 operator()(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3) const {
    uint32_t a = k0, b = k1;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
      if (r) { a += 0x9E3779B9u; b += 0xBB67AE85u; }
      const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
      const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
      const uint32_t n0 = hi1 ^ c1 ^ a, n2 = hi0 ^ c3 ^ b;
      c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    return make_uint4(c0, c1, c2, c3);
  }
};

// (2 (w >> 9) + 1) 2^-24: uniform on (0, 1), exact in FP32 and FP64
__device__ __forceinline__ double unif(uint32_t w) { return ((double)(w >> 9) + 0.5) * 0x1p-23; }

struct SimArgs {
  int T, F, N, m, L;
  float max_doppler, snr_lo, snr_hi;
  uint32_t k0, k1;
  int64_t first_slot;
  float2* y;
  uint8_t* bits;
  float* noise_var;
  float sqrt_p[SIM_LMAX];       // sqrt of the tap powers
};

// Gray QAM axis level of k bits c_0 .. c_{k-1} (c_0 the sign): s_0 (2^{k-1} - s_1 (2^{k-2} - ...
// (2 - s_{k-1}))), s_i = 1 - 2 c_i -- the nested form of the NR square constellations
__device__ __forceinline__ int qam_level(uint32_t w, int first, int k) {
  int tail = 1;
  for (int i = k - 1; i >= 1; --i) {
    const int s = 1 - 2 * (int)((w >> (first + 2 * i)) & 1u);
    tail = (1 << (k - i)) - s * tail;
  }
  return (1 - 2 * (int)((w >> first) & 1u)) * tail;
}

__global__ void __launch_bounds__(256) simulate_kernel(SimArgs a) {
  __shared__ float2 g[SIM_LMAX * SIM_NMAX];
  const int64_t slot = a.first_slot + blockIdx.y;
  const int t = blockIdx.x;
  const Philox ph{a.k0, a.k1};
  const uint32_t sl = (uint32_t)(slot & 0xffffffffu);
  const uint4 sp = ph(sl, 1u, 0u, 0u);
  const double fd = unif(sp.x) * (double)a.max_doppler;
  const double snr_db = (double)a.snr_lo + unif(sp.y) * (double)(a.snr_hi - a.snr_lo);
  const double nv = pow(10.0, -snr_db / 10.0);
  if (threadIdx.x == 0 && t == 0 && a.noise_var) a.noise_var[blockIdx.y] = (float)nv;
  // channel taps of this symbol, one thread per (tap, antenna)
  for (int i = threadIdx.x; i < a.L * a.N; i += blockDim.x) {
    double re = 0.0, im = 0.0;
    for (int s = 0; s < SIM_PATHS; ++s) {
      const uint4 w = ph(sl, 4u, (uint32_t)(i * SIM_PATHS + s), 0u);
      const double ca = cospi(2.0 * unif(w.x));
      const double arg = 2.0 * fd * SIM_SYMBOL_PERIOD_S * t * ca + 2.0 * unif(w.y);  // in units of pi
      double sn, cs;
      sincospi(arg, &sn, &cs);
      re += cs;
      im += sn;
    }
    const double sc = 1.0 / sqrt((double)SIM_PATHS);
    g[i] = make_float2((float)(re * sc), (float)(im * sc));
  }
  __syncthreads();
  const double nsd = sqrt(nv);
  const double qn = 1.0 / sqrt(2.0 * ((double)(1 << a.m) - 1.0) / 3.0);
  const int kb = a.m / 2;
  for (int f = threadIdx.x; f < a.F; f += blockDim.x) {
    const int64_t re_idx = (int64_t)blockIdx.y * a.T * a.F + (int64_t)t * a.F + f;
    const uint32_t idx = (uint32_t)(t * a.F + f);
    const uint32_t wb = ph(sl, 2u, idx, 0u).x;
    for (int i = 0; i < a.m; ++i) a.bits[re_idx * a.m + i] = (uint8_t)((wb >> i) & 1u);
    double xr, xi;
    if ((t == PILOT_T0 || t == PILOT_T1) && (f & 1) == 0) {
      xr = xi = 0.70710678118654752;
    } else {  // even bits set the in-phase level, odd bits the quadrature
      xr = qam_level(wb, 0, kb) * qn;
      xi = qam_level(wb, 1, kb) * qn;
    }
    // tap phases exp(-j 2 pi f df tau_l)
    float2 e[SIM_LMAX];
    for (int l = 0; l < a.L; ++l) {
      double x = (double)f * SIM_SUBCARRIER_HZ * (l * SIM_TAP_SPACING_S);
      x -= floor(x);
      double sn, cs;
      sincospi(2.0 * x, &sn, &cs);
      e[l] = make_float2((float)(cs * a.sqrt_p[l]), (float)(-sn * a.sqrt_p[l]));
    }
    for (int n = 0; n < a.N; ++n) {
      double hr = 0.0, hi = 0.0;
      for (int l = 0; l < a.L; ++l) {
        const float2 gv = g[l * a.N + n];
        hr += (double)gv.x * e[l].x - (double)gv.y * e[l].y;
        hi += (double)gv.x * e[l].y + (double)gv.y * e[l].x;
      }
      const uint4 wn = ph(sl, 3u, idx * (uint32_t)a.N + (uint32_t)n, 0u);
      const double r = sqrt(-log(unif(wn.x))) * nsd;
      double sn, cs;
      sincospi(2.0 * unif(wn.y), &sn, &cs);
      const double yr = hr * xr - hi * xi + r * cs;
      const double yi = hr * xi + hi * xr + r * sn;
      a.y[re_idx * a.N + n] = make_float2((float)yr, (float)yi);
    }
  }
}

}  // namespace conet

using namespace conet;

extern "C" conet_status conet_simulate(const conet_sim_config* cfg, int64_t first_slot, int32_t B, float* y,
                                       uint8_t* bits, float* noise_var, void* stream) {
  if (!cfg) return fail(CONET_EINVAL, "null config");
  if (B == 0) return CONET_OK;
  if (!y || !bits) return fail(CONET_EINVAL, "null output buffer");
  if (B < 0 || B > 65535 || cfg->F < 1 || cfg->T < PILOT_T1 + 1 || cfg->T > TMAX)
    return fail(CONET_ESHAPE, "need 1 <= B <= 65535, F >= 1, 12 <= T <= 14");
  if (cfg->n_rx < 1 || cfg->n_rx > SIM_NMAX) return fail(CONET_EINVAL, "n_rx must be 1..%d", SIM_NMAX);
  if (cfg->n_taps < 1 || cfg->n_taps > SIM_LMAX) return fail(CONET_EINVAL, "n_taps must be 1..%d", SIM_LMAX);
  if (cfg->bits_per_symbol < 2 || cfg->bits_per_symbol > 8 || (cfg->bits_per_symbol & 1))
    return fail(CONET_EINVAL, "square QAM needs 2, 4, 6 or 8 bits per symbol");
  if (!(cfg->max_doppler_hz >= 0.f) || !(cfg->snr_hi_db >= cfg->snr_lo_db))
    return fail(CONET_EINVAL, "need max_doppler_hz >= 0 and snr_hi_db >= snr_lo_db");
  if ((int64_t)cfg->T * cfg->F * cfg->n_rx > 0xffffffffLL) return fail(CONET_ESHAPE, "grid too large");
  SimArgs a = {};
  a.T = cfg->T; a.F = cfg->F; a.N = cfg->n_rx; a.m = cfg->bits_per_symbol; a.L = cfg->n_taps;
  a.max_doppler = cfg->max_doppler_hz; a.snr_lo = cfg->snr_lo_db; a.snr_hi = cfg->snr_hi_db;
  a.k0 = (uint32_t)(cfg->seed & 0xffffffffu);
  a.k1 = (uint32_t)(cfg->seed >> 32);
  a.first_slot = first_slot;
  a.y = reinterpret_cast<float2*>(y);
  a.bits = bits;
  a.noise_var = noise_var;
  // exponential power delay profile, normalised to unit total power
  double ps[SIM_LMAX], tot = 0.0;
  for (int l = 0; l < a.L; ++l) { ps[l] = std::exp(-(l * SIM_TAP_SPACING_S) / SIM_PDP_DECAY_S); tot += ps[l]; }
  for (int l = 0; l < a.L; ++l) a.sqrt_p[l] = (float)std::sqrt(ps[l] / tot);
  hipLaunchKernelGGL(simulate_kernel, dim3(cfg->T, B), dim3(256), 0, (hipStream_t)stream, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "simulate launch");
  return CONET_OK;
}
