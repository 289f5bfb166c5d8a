// Device-side definitions shared by the CoNet-Rx gfx950 kernels.
//
// Arithmetic policies bind one MFMA instruction to the element types it reads and
// the layout in which a lane supplies its operands. Every policy reads its B operand
// (activations) from LDS in 16-byte "chunks" of consecutive channels of one tap, so a
// 3x3 conv becomes an implicit GEMM whose K index runs over (tap, channel chunk).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace conet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int KMAX = 8;          // most branches one launch can address
constexpr int TMAX = 14;         // OFDM symbols per TTI held in one tile
constexpr int TROWS = TMAX + 2;  // plus the zero halo rows above and below
constexpr float E4M3_MAX = 448.0f;

typedef uint8_t fp8;             // OCP e4m3fn bit pattern

// ---------------------------------------------------------------- scalar converts
__device__ __forceinline__ float to_f(float v) { return v; }
__device__ __forceinline__ float to_f(__bf16 v) { return (float)v; }

// RNE float -> bf16 (the hardware conversion rounds to nearest even).
__device__ __forceinline__ __bf16 f2bf(float v) { return (__bf16)v; }

// Saturating RNE float -> e4m3fn: clamp to +-448, then the hardware conversion.
__device__ __forceinline__ uint32_t pack4_e4m3(float a, float b, float c, float d) {
  a = fminf(fmaxf(a, -E4M3_MAX), E4M3_MAX);
  b = fminf(fmaxf(b, -E4M3_MAX), E4M3_MAX);
  c = fminf(fmaxf(c, -E4M3_MAX), E4M3_MAX);
  d = fminf(fmaxf(d, -E4M3_MAX), E4M3_MAX);
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);
  return (uint32_t)w;
}

// ---------------------------------------------------------------- policies
// VEC: operand elements per 16-byte chunk. CPL: chunks one lane supplies per MFMA.
// Acc: accumulator / epilogue type. Act: residual-stream storage type. Hid: storage
// type of the block's middle activation (the second conv's operand).

struct ArithF32 {
  using Op = float; using Acc = float; using AccV = f32x4; using Act = float; using Hid = float;
  static constexpr int VEC = 4, CPL = 1;
  static constexpr bool QUANT = false;
  __device__ __forceinline__ static AccV mma(const i32x4* a, const i32x4* b, AccV c) {
    const float* fa = reinterpret_cast<const float*>(a);
    const float* fb = reinterpret_cast<const float*>(b);
#pragma unroll
    for (int q = 0; q < 4; ++q) c = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[q], fb[q], c, 0, 0, 0);
    return c;
  }
};

struct ArithBF16 {
  using Op = __bf16; using Acc = float; using AccV = f32x4; using Act = __bf16; using Hid = __bf16;
  static constexpr int VEC = 8, CPL = 1;
  static constexpr bool QUANT = false;
  __device__ __forceinline__ static AccV mma(const i32x4* a, const i32x4* b, AccV c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[0]),
                                                   __builtin_bit_cast(bf16x8, b[0]), c, 0, 0, 0);
  }
};

struct ArithFP8 {
  using Op = fp8; using Acc = float; using AccV = f32x4; using Act = __bf16; using Hid = fp8;
  static constexpr int VEC = 16, CPL = 2;
  static constexpr bool QUANT = true;
  __device__ __forceinline__ static AccV mma(const i32x4* a, const i32x4* b, AccV c) {
    i32x8 av, bv;
#pragma unroll
    for (int i = 0; i < 4; ++i) { av[i] = a[0][i]; av[4 + i] = a[1][i]; bv[i] = b[0][i]; bv[4 + i] = b[1][i]; }
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, c, 0, 0, 0, 0, 0, 0);
  }
};

// ---------------------------------------------------------------- LS channel estimate
// Pilots: OFDM symbols 2 and 11, even subcarriers, value p = (1 + j)/sqrt(2). Shared by the
// featuriser and the input conv's grid staging, so both form bit-identical features.
constexpr int PILOT_T0 = 2, PILOT_T1 = 11;

// y / p = y conj(p) / |p|^2 = ((a + b) + j (b - a)) / sqrt(2)
__device__ __forceinline__ float2 div_pilot(float2 y) {
  const float r = 0.70710678118654752f;
  return make_float2((y.x + y.y) * r, (y.y - y.x) * r);
}

// LS estimate on one pilot symbol at subcarrier f of one antenna (row: pointer to that
// antenna's sample at subcarrier 0 of the symbol, stride floats2 per subcarrier): y / p on
// even f, the mean of the two even neighbours on odd f, the left neighbour on a last odd f.
__device__ __forceinline__ float2 pilot_row_estimate(const float2* __restrict__ row, int64_t stride, int f, int F) {
  if ((f & 1) == 0) return div_pilot(row[(int64_t)f * stride]);
  const float2 l = div_pilot(row[(int64_t)(f - 1) * stride]);
  if (f + 1 >= F) return l;
  const float2 r = div_pilot(row[(int64_t)(f + 1) * stride]);
  return make_float2(0.5f * (l.x + r.x), 0.5f * (l.y + r.y));
}

// Every symbol t on the line through the two pilot symbols: h0 + (t - 2) / 9 (h1 - h0).
__device__ __forceinline__ float2 interp_symbol(float2 h0, float2 h1, int t) {
  const float w = (float)(t - PILOT_T0) / (float)(PILOT_T1 - PILOT_T0);
  return make_float2(fmaf(w, h1.x - h0.x, h0.x), fmaf(w, h1.y - h0.y, h0.y));
}

// ---------------------------------------------------------------- tile geometry
// A tile is one slot, all of its T <= 14 OFDM symbols and TW consecutive subcarriers.
struct TileDesc {
  int64_t re_base;  // index of RE (t = 0, f = 0) of the tile's slot in the packed tensor
  int32_t F;        // subcarriers of that slot
  int32_t f0;       // first subcarrier of the tile
};

}  // namespace conet
