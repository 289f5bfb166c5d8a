// Block and fusion variants of CoNet-Rx on gfx950.
//
// Depthwise-separable residual block (Sec. II-A: each conv of a block may be a depthwise 3x3
// filter followed by a 1x1 conv). One work-group runs both separable convs of one block of
// one branch for a tile of DS_TW subcarriers x all T symbols of one slot; h never leaves LDS:
//   stage pre(x) over DS_TW + 4 columns (rounded to the operand type, zero outside the slot)
//   -> depthwise 1 over DS_TW + 2 columns (VALU: FP32 sums of 9 products, rounded as the
//      1x1 conv's operand, formed in the registers that feed the MFMA) -> 1x1 conv 1 on MFMA
//   -> bias, affine, ReLU, zero outside the slot = h (to LDS) -> depthwise 2 over DS_TW
//      columns, again straight into the B fragments -> 1x1 conv 2 on MFMA -> + bias + x.
// Per RE and branch the block reads and writes C activations (plus a 4-column halo) for
// 2 (18 C + 2 C^2) FLOPs: 73 FLOP per HBM byte at C = 64 in BF16, far below the ratio of
// the MI355X's BF16 MFMA rate to its HBM bandwidth, so the kernel is HBM-bound.
//
// Fusion epilogue: one pass per RE for fusions that no block kernel folds in (fusion by
// concatenation, Sec. III, after any block; every fusion after separable blocks). P comes
// from the stored branch outputs -- their product or sum, or the 1x1 projection of their
// concatenation (MFMA) -- then LayerNorm (or the folded BatchNorm affine), the fused
// activation, Example II feedback into the support outputs, and the head.
#include <hip/hip_runtime.h>

#include <cstring>

#include "conet_common.h"
#include "conet_kernels.h"
#include "conet_model.h"

namespace conet {

// ---------------------------------------------------------------- 1x1 filter packing
// Fragments of the 16x16 MFMAs for a 1x1 conv W[cout][cin]: [s][ot][lane] x 16 bytes, lane
// l supplying row o = 16 ot + l % 16 and the VEC input channels of chunk 4 s + l / 16 (the
// K step s covers 4 VEC channels). The accumulator of lane l then holds output channels
// 16 ot + 4 (l / 16) + q, q = 0..3, of the RE in column l % 16.
static int vec_of(int dtype) { return dtype == DT_F32 ? 4 : 8; }

size_t packed_bytes_1x1(int dtype, int cin, int cout) {
  const int ns = cin / (4 * vec_of(dtype));
  return (size_t)ns * (cout / 16) * 64 * 16;
}

void pack_1x1(int dtype, int cin, int cout, const float* W, uint8_t* dst) {
  const int vec = vec_of(dtype), ns = cin / (4 * vec), NOT = cout / 16;
  for (int s = 0; s < ns; ++s)
    for (int ot = 0; ot < NOT; ++ot)
      for (int lane = 0; lane < 64; ++lane) {
        uint8_t* out = dst + (((size_t)s * NOT + ot) * 64 + lane) * 16;
        const int o = 16 * ot + (lane & 15), c0 = (4 * s + (lane >> 4)) * vec;
        for (int e = 0; e < vec; ++e) {
          const float w = W[(size_t)o * cin + c0 + e];
          if (dtype == DT_F32) {
            memcpy(out + 4 * e, &w, 4);
          } else {
            const uint16_t b = bf16_bits(w);
            memcpy(out + 2 * e, &b, 2);
          }
        }
      }
}

bool ds_supported(int dtype, int C) { return (dtype == DT_F32 || dtype == DT_BF16) && (C == 32 || C == 64); }
bool concat_supported(int dtype, int C, int K) { return ds_supported(dtype, C) && K >= 1 && K <= 4; }

// ---------------------------------------------------------------- separable block
// Waves per work-group: 8, so that with two work-groups per CU every SIMD holds four waves to
// hide the staging and LDS latencies (the block is latency-bound at four waves per work-group:
// 45 % of wave cycles waited on memory counters).
constexpr int DS_NW = 8;

template <class A, int C>
struct DsShape {
  using Op = typename A::Op;
  static constexpr int VEC = A::VEC;                  // operand elements per 16 bytes
  static constexpr int CH = C / VEC;                  // 16-byte chunks per position
  static constexpr int PITCH = C * (int)sizeof(Op) + 16;  // bytes per staged position
  static constexpr int W0 = DS_TW + 4;                // columns of pre(x): the tile +- 2
  static constexpr int W1 = DS_TW + 2;                // columns of d1 and h: the tile +- 1
  static constexpr int PRE = TMAX * W0 * PITCH;       // pre(x)
  static constexpr int MID = TMAX * W1 * PITCH;       // h
  static constexpr int LDS = PRE + MID;
  static constexpr int NT = DS_NW * 64;               // threads per work-group
  static constexpr int NSTAGE = (TMAX * W0 * CH + NT - 1) / NT;  // staging items per thread
  static constexpr int NOT = C / 16;
  static constexpr int NS = C / (4 * VEC);            // K steps of a 1x1 conv
  static constexpr int MT = (16 + DS_NW - 1) / DS_NW;  // RE tiles of 16 per wave and conv (<= 16 tiles)
  using AccTile = typename A::AccV[MT][NOT];
  static_assert(C % (4 * VEC) == 0, "1x1 conv K steps must be whole");
  static_assert(LDS <= 160 * 1024, "LDS budget");
};

template <class A>
__device__ __forceinline__ void chunk_to_f(const i32x4& raw, float* f) {
  using Op = typename A::Op;
  const Op* e = reinterpret_cast<const Op*>(&raw);
#pragma unroll
  for (int j = 0; j < A::VEC; ++j) f[j] = (float)e[j];
}

template <class A>
__device__ __forceinline__ i32x4 f_to_chunk(const float* f) {
  using Op = typename A::Op;
  i32x4 raw;
  Op* e = reinterpret_cast<Op*>(&raw);
#pragma unroll
  for (int j = 0; j < A::VEC; ++j) e[j] = (Op)f[j];  // BF16: round to nearest even
  return raw;
}

// One separable conv over the n_cols-wide region of positions (t, col), t < T: the depthwise
// 3x3 filter (output column col reads input columns col .. col + 2 of `in`, which is two
// columns wider; rows outside [0, T) read as zero) feeds the 1x1 conv's B fragments straight
// from registers -- each depthwise output is one lane's operand chunk and is used once -- so
// it is never stored. Per K step s the lane's chunk is 4 s + l / 16; its 9 x VEC taps are
// loaded once per step. acc[mt][ot] covers RE tiles wave + DS_NW mt (tiles past the region
// compute position 0 and are discarded).
template <class A, int C>
__device__ __forceinline__ void separable(typename DsShape<A, C>::AccTile& acc, const uint8_t* in, int in_w,
                                          int n_cols, int T, const float* __restrict__ dw,
                                          const i32x4* __restrict__ wp) {
  using S = DsShape<A, C>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4;
  const int n_pos = T * n_cols;
  int tt0[S::MT], cc0[S::MT];
#pragma unroll
  for (int mt = 0; mt < S::MT; ++mt) {
    int pos = (wave + DS_NW * mt) * 16 + (lane & 15);
    if (pos >= n_pos) pos = 0;
    tt0[mt] = pos / n_cols;
    cc0[mt] = pos - tt0[mt] * n_cols;
#pragma unroll
    for (int ot = 0; ot < S::NOT; ++ot) acc[mt][ot] = typename A::AccV{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int s = 0; s < S::NS; ++s) {
    const int chunk = 4 * s + g;
    i32x4 a[S::NOT];
#pragma unroll
    for (int ot = 0; ot < S::NOT; ++ot) a[ot] = wp[(s * S::NOT + ot) * 64 + lane];
    float d[S::MT][A::VEC];
#pragma unroll
    for (int mt = 0; mt < S::MT; ++mt)
#pragma unroll
      for (int j = 0; j < A::VEC; ++j) d[mt][j] = 0.f;
    // one filter row (3 taps) at a time, shared by the lane's RE tiles: fewer live registers
#pragma unroll
    for (int dt = -1; dt <= 1; ++dt) {
      float w[3][A::VEC];
#pragma unroll
      for (int df = 0; df < 3; ++df)
#pragma unroll
        for (int j = 0; j < A::VEC; ++j) w[df][j] = dw[((dt + 1) * 3 + df) * C + chunk * A::VEC + j];
#pragma unroll
      for (int mt = 0; mt < S::MT; ++mt) {
        const int tt = tt0[mt] + dt;
        if (tt < 0 || tt >= T) continue;
#pragma unroll
        for (int df = 0; df < 3; ++df) {
          float v[A::VEC];
          chunk_to_f<A>(*reinterpret_cast<const i32x4*>(in + (tt * in_w + cc0[mt] + df) * S::PITCH + chunk * 16), v);
#pragma unroll
          for (int j = 0; j < A::VEC; ++j) d[mt][j] = fmaf(w[df][j], v[j], d[mt][j]);
        }
      }
    }
#pragma unroll
    for (int mt = 0; mt < S::MT; ++mt) {
      const i32x4 b = f_to_chunk<A>(d[mt]);  // the 1x1 conv's operand, rounded
#pragma unroll
      for (int ot = 0; ot < S::NOT; ++ot) acc[mt][ot] = A::mma(&a[ot], &b, acc[mt][ot]);
    }
  }
}

__device__ __forceinline__ TileDesc ds_tile(const DsArgs& a, int bid) {
  if (a.tiles) return a.tiles[bid];
  TileDesc d;
  const int b = bid / a.tiles_per_slot;
  d.re_base = (int64_t)b * a.T * a.F;
  d.F = a.F;
  d.f0 = (bid - b * a.tiles_per_slot) * DS_TW;
  return d;
}

// two work-groups per CU where the LDS allows it (not at C = 64 in FP32: 149 KB); the second
// launch bound is the waves per SIMD that implies, which caps the registers per lane
template <class A, int C>
__global__ void __launch_bounds__(DS_NW * 64, (DsShape<A, C>::LDS <= 80 * 1024 ? 2 : 1) * DS_NW / 4)
    ds_block_kernel(DsArgs args) {
  using S = DsShape<A, C>;
  using Op = typename A::Op;
  __shared__ __attribute__((aligned(16))) uint8_t lds[S::LDS];
  uint8_t* pre = lds;
  uint8_t* mid = lds + S::PRE;
  const int k = blockIdx.y + args.k_off;
  const TileDesc td = ds_tile(args, blockIdx.x);
  const int T = args.T, lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4;
  const Op* __restrict__ x = reinterpret_cast<const Op*>(args.x[k]);

  // pre(x) = ReLU(s0 x + o0), or ReLU(x) in a main block after a fusion; zero outside the slot.
  // A thread keeps one channel chunk (its prologue parameters in registers) and issues all of
  // its loads before converting any, so their latencies overlap.
  {
    const int c16 = threadIdx.x % S::CH;
    const bool aff = args.pre_s[k] != nullptr;
    float sv[A::VEC], ov[A::VEC];
#pragma unroll
    for (int j = 0; j < A::VEC; ++j) {
      sv[j] = aff ? args.pre_s[k][c16 * A::VEC + j] : 1.f;
      ov[j] = aff ? args.pre_o[k][c16 * A::VEC + j] : 0.f;
    }
    i32x4 raw[S::NSTAGE];
#pragma unroll
    for (int it = 0; it < S::NSTAGE; ++it) {
      const int i = threadIdx.x + it * S::NT;
      const int pos = i / S::CH, col = pos % S::W0, t = pos / S::W0;
      const int f = td.f0 - 2 + col;
      raw[it] = i32x4{0, 0, 0, 0};
      if (i < TMAX * S::W0 * S::CH && t < T && f >= 0 && f < td.F)
        raw[it] = *reinterpret_cast<const i32x4*>(x + (td.re_base + (int64_t)t * td.F + f) * C + c16 * A::VEC);
    }
#pragma unroll
    for (int it = 0; it < S::NSTAGE; ++it) {
      const int i = threadIdx.x + it * S::NT;
      if (i >= TMAX * S::W0 * S::CH) break;
      const int pos = i / S::CH, col = pos % S::W0, t = pos / S::W0;
      const int f = td.f0 - 2 + col;
      i32x4 v = {0, 0, 0, 0};
      if (t < T && f >= 0 && f < td.F) {
        float e[A::VEC];
        chunk_to_f<A>(raw[it], e);
#pragma unroll
        for (int j = 0; j < A::VEC; ++j) e[j] = fmaxf(fmaf(sv[j], e[j], ov[j]), 0.f);
        v = f_to_chunk<A>(e);
      }
      *reinterpret_cast<i32x4*>(pre + pos * S::PITCH + c16 * 16) = v;
    }
  }
  __syncthreads();

  typename S::AccTile acc;
  separable<A, C>(acc, pre, S::W0, S::W1, T, args.dw1[k], reinterpret_cast<const i32x4*>(args.pw1[k]));
  {
    const float* b1 = args.b1[k];
    const float* s1 = args.post_s[k];
    const float* o1 = args.post_o[k];
#pragma unroll
    for (int mt = 0; mt < S::MT; ++mt) {
      const int pos = (wave + DS_NW * mt) * 16 + (lane & 15);
      if (pos >= T * S::W1) continue;
      const int col = pos % S::W1;
      const int f = td.f0 - 1 + col;
      const bool in_slot = f >= 0 && f < td.F;
#pragma unroll
      for (int ot = 0; ot < S::NOT; ++ot) {
        Op hv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int o = 16 * ot + 4 * g + q;
          const float z = fmaf(s1[o], acc[mt][ot][q] + b1[o], o1[o]);
          hv[q] = (Op)(in_slot ? fmaxf(z, 0.f) : 0.f);
        }
        Op* dst = reinterpret_cast<Op*>(mid + pos * S::PITCH) + 16 * ot + 4 * g;
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = hv[q];
      }
    }
  }
  __syncthreads();
  separable<A, C>(acc, mid, S::W1, DS_TW, T, args.dw2[k], reinterpret_cast<const i32x4*>(args.pw2[k]));
  // Epilogue through LDS: conv 2 + bias goes to an FP32 tile [position][C] (every wave has read
  // h, so the LDS is free), then each thread adds x and stores 8 consecutive channels of one
  // RE, so the residual reads and the output writes are contiguous 16-byte accesses.
  constexpr int OP = C * 4 + 16;
  static_assert(TMAX * DS_TW * OP <= S::LDS, "output tile must fit the LDS");
  __syncthreads();
  {
    const float* b2 = args.b2[k];
#pragma unroll
    for (int mt = 0; mt < S::MT; ++mt) {
      const int pos = (wave + DS_NW * mt) * 16 + (lane & 15);
      if (pos >= T * DS_TW) continue;
#pragma unroll
      for (int ot = 0; ot < S::NOT; ++ot) {
        const int o0 = 16 * ot + 4 * g;
        *reinterpret_cast<float4*>(lds + pos * OP + o0 * 4) =
            make_float4(acc[mt][ot][0] + b2[o0], acc[mt][ot][1] + b2[o0 + 1], acc[mt][ot][2] + b2[o0 + 2],
                        acc[mt][ot][3] + b2[o0 + 3]);
      }
    }
  }
  __syncthreads();
  {
    constexpr int C8 = C / 8;
    const bool f32 = args.out_f32[k] != 0;
    for (int i = threadIdx.x; i < T * DS_TW * C8; i += S::NT) {
      const int pos = i / C8, c0 = (i - pos * C8) * 8;
      const int t = pos / DS_TW, f = td.f0 + pos % DS_TW;
      if (f >= td.F) continue;
      const int64_t re = td.re_base + (int64_t)t * td.F + f;
      const float4 lo = *reinterpret_cast<const float4*>(lds + pos * OP + c0 * 4);
      const float4 hi = *reinterpret_cast<const float4*>(lds + pos * OP + c0 * 4 + 16);
      float v[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
      const i32x4* xp = reinterpret_cast<const i32x4*>(x + re * C + c0);
      float xv[8];
      if constexpr (sizeof(Op) == 2) {
        chunk_to_f<A>(xp[0], xv);
      } else {
        chunk_to_f<A>(xp[0], xv);
        chunk_to_f<A>(xp[1], xv + 4);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] += xv[j];
      if (f32) {
        float4* dst = reinterpret_cast<float4*>(reinterpret_cast<float*>(args.out[k]) + re * C + c0);
        dst[0] = make_float4(v[0], v[1], v[2], v[3]);
        dst[1] = make_float4(v[4], v[5], v[6], v[7]);
      } else if constexpr (sizeof(Op) == 2) {
        *reinterpret_cast<i32x4*>(reinterpret_cast<Op*>(args.out[k]) + re * C + c0) = f_to_chunk<A>(v);
      } else {
        i32x4* dst = reinterpret_cast<i32x4*>(reinterpret_cast<Op*>(args.out[k]) + re * C + c0);
        dst[0] = f_to_chunk<A>(v);
        dst[1] = f_to_chunk<A>(v + 4);
      }
    }
  }
}

template <class A, int C>
static hipError_t launch_ds_t(DsArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  a.tw = DS_TW;
  hipLaunchKernelGGL((ds_block_kernel<A, C>), dim3(n_tiles, grid_y), dim3(DS_NW * 64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ds_block(int dtype, int C, DsArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  if (n_tiles <= 0 || grid_y <= 0) return hipSuccess;
  if (dtype == DT_BF16 && C == 64) return launch_ds_t<ArithBF16, 64>(a, n_tiles, grid_y, s);
  if (dtype == DT_BF16 && C == 32) return launch_ds_t<ArithBF16, 32>(a, n_tiles, grid_y, s);
  if (dtype == DT_F32 && C == 64) return launch_ds_t<ArithF32, 64>(a, n_tiles, grid_y, s);
  if (dtype == DT_F32 && C == 32) return launch_ds_t<ArithF32, 32>(a, n_tiles, grid_y, s);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- fusion epilogue
// 4 waves of 16 REs per work-group; lane l holds channels 16 ot + 4 (l / 16) + q of RE l % 16
// (the MFMA accumulator layout), so a RE's C channels sit in 4 lanes 16 apart.
template <class A>
__device__ __forceinline__ void load4(const void* base, bool f32, int64_t idx, float* v) {
  if (f32) {
    const float4 w = *reinterpret_cast<const float4*>(reinterpret_cast<const float*>(base) + idx);
    v[0] = w.x; v[1] = w.y; v[2] = w.z; v[3] = w.w;
  } else {
    const typename A::Op* p = reinterpret_cast<const typename A::Op*>(base) + idx;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (float)p[q];
  }
}

template <class A>
__device__ __forceinline__ void store4(void* base, int64_t idx, const float* v) {
  typename A::Op* p = reinterpret_cast<typename A::Op*>(base) + idx;
#pragma unroll
  for (int q = 0; q < 4; ++q) p[q] = (typename A::Op)v[q];
}

__device__ __forceinline__ float sum_over_groups(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

template <class A, int C, int MODE>
__global__ void __launch_bounds__(256) fuse_epilogue_kernel(FuseArgs a) {
  using Op = typename A::Op;
  constexpr int NOT = C / 16;
  constexpr bool act_f32 = sizeof(Op) == 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4;
  const int64_t r = ((int64_t)blockIdx.x * 4 + wave) * 16 + (lane & 15);
  const bool ok = r < a.n_re;
  const int64_t rr = ok ? r : 0;  // rows past the end read row 0 and store nothing
  float P[NOT][4];
  if constexpr (MODE == EPI_CONCAT) {
    typename A::AccV acc[NOT];
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot) acc[ot] = typename A::AccV{0.f, 0.f, 0.f, 0.f};
    const i32x4* __restrict__ wp = reinterpret_cast<const i32x4*>(a.wcat);
    const int ns = a.K * C / (4 * A::VEC);
    for (int s = 0; s < ns; ++s) {
      const int chunk = 4 * s + g;
      const int kb = chunk * A::VEC / C, ch = chunk * A::VEC - kb * C;
      const Op* src = reinterpret_cast<const Op*>(kb == 0 ? a.main : a.sup[kb]);
      const i32x4 b = *reinterpret_cast<const i32x4*>(src + rr * C + ch);
#pragma unroll
      for (int ot = 0; ot < NOT; ++ot) {
        const i32x4 w = wp[(s * NOT + ot) * 64 + lane];
        acc[ot] = A::mma(&w, &b, acc[ot]);
      }
    }
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int q = 0; q < 4; ++q) P[ot][q] = acc[ot][q] + a.bcat[16 * ot + 4 * g + q];
  } else {
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot) {
      const int o0 = 16 * ot + 4 * g;
      load4<A>(a.main, a.main_f32 || act_f32, rr * C + o0, P[ot]);
      if constexpr (MODE == EPI_PRODUCT || MODE == EPI_SUM) {
        for (int k = 1; k < a.K; ++k) {
          float v[4];
          load4<A>(a.sup[k], act_f32, rr * C + o0, v);
#pragma unroll
          for (int q = 0; q < 4; ++q) P[ot][q] = MODE == EPI_SUM ? P[ot][q] + v[q] : P[ot][q] * v[q];
        }
      }
    }
  }
  float Av[NOT][4];
  if constexpr (MODE == EPI_NONE) {
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int q = 0; q < 4; ++q) Av[ot][q] = P[ot][q];
  } else if (a.norm_affine) {
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = 16 * ot + 4 * g + q;
        Av[ot][q] = fmaf(a.gamma[o], P[ot][q], a.beta[o]);
      }
  } else {  // LayerNorm over the C channels of the RE
    float s = 0.f;
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int q = 0; q < 4; ++q) s += P[ot][q];
    const float mu = sum_over_groups(s) / (float)C;
    float v = 0.f;
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float d = P[ot][q] - mu;
        v = fmaf(d, d, v);
      }
    const float inv = 1.0f / sqrtf(sum_over_groups(v) / (float)C + a.eps);
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = 16 * ot + 4 * g + q;
        Av[ot][q] = fmaf(a.gamma[o], (P[ot][q] - mu) * inv, a.beta[o]);
      }
  }
  if (ok && a.out) {
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot) store4<A>(a.out, r * C + 16 * ot + 4 * g, Av[ot]);
  }
  if (ok && a.feedback) {  // support k continues from its stored output plus the fused activation
    for (int k = 1; k < a.K; ++k)
#pragma unroll
      for (int ot = 0; ot < NOT; ++ot) {
        const int64_t idx = r * C + 16 * ot + 4 * g;
        float v[4];
        load4<A>(a.sup[k], act_f32, idx, v);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] += Av[ot][q];
        store4<A>(a.sup[k], idx, v);
      }
  }
  if (a.llr) {  // head on the unrounded activation
    for (int j = 0; j < a.m; ++j) {
      float s = 0.f;
#pragma unroll
      for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
        for (int q = 0; q < 4; ++q) s = fmaf(a.Wh[j * C + 16 * ot + 4 * g + q], Av[ot][q], s);
      s = sum_over_groups(s);
      if (ok && g == 0) a.llr[r * a.m + j] = s + a.bh[j];
    }
  }
}

template <class A, int C>
static hipError_t launch_fuse_t(int mode, FuseArgs& a, unsigned blocks, hipStream_t s) {
  switch (mode) {
    case EPI_NONE: hipLaunchKernelGGL((fuse_epilogue_kernel<A, C, EPI_NONE>), dim3(blocks), dim3(256), 0, s, a); break;
    case EPI_PRODUCT: hipLaunchKernelGGL((fuse_epilogue_kernel<A, C, EPI_PRODUCT>), dim3(blocks), dim3(256), 0, s, a); break;
    case EPI_SUM: hipLaunchKernelGGL((fuse_epilogue_kernel<A, C, EPI_SUM>), dim3(blocks), dim3(256), 0, s, a); break;
    case EPI_CONCAT: hipLaunchKernelGGL((fuse_epilogue_kernel<A, C, EPI_CONCAT>), dim3(blocks), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fuse_epilogue(int dtype, int C, int mode, FuseArgs& a, hipStream_t s) {
  const int64_t blocks = (a.n_re + 63) / 64;
  if (blocks <= 0) return hipSuccess;
  if (blocks > 0x7fffffff) return hipErrorInvalidValue;
  if (dtype == DT_BF16 && C == 64) return launch_fuse_t<ArithBF16, 64>(mode, a, (unsigned)blocks, s);
  if (dtype == DT_BF16 && C == 32) return launch_fuse_t<ArithBF16, 32>(mode, a, (unsigned)blocks, s);
  if (dtype == DT_F32 && C == 64) return launch_fuse_t<ArithF32, 64>(mode, a, (unsigned)blocks, s);
  if (dtype == DT_F32 && C == 32) return launch_fuse_t<ArithF32, 32>(mode, a, (unsigned)blocks, s);
  return hipErrorInvalidValue;
}

}  // namespace conet
