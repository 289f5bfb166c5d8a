// 3x3 implicit-GEMM convolution kernels of the CoNet-Rx forward pass (gfx950).
//
// One work-group owns one tile: a slot, all of its T <= 14 OFDM symbols and TW
// consecutive subcarriers. The tile's input (with a one-RE zero halo on every side,
// padding taken inside the slot) is staged once into LDS in the MFMA operand type;
// the optional pre-activation prologue (affine + ReLU, or ReLU) and FP8 quantisation
// are applied during staging. Each wave then runs the GEMM
//     D^T[o, re] = sum_k W[o, k] * X^T[k, re],   k = (tap, channel)
// on 16x16 MFMA tiles: the A operand is the filter, pre-packed on the host in the
// exact per-lane fragment order (one coalesced 16-byte load per lane), and the B
// operand is read from LDS as 16-byte chunks of consecutive channels at the
// tap-shifted position. The epilogue works on FP32 accumulators in registers:
// bias, per-channel affine, ReLU, residual add, the K-way product fusion with the
// per-RE channel LayerNorm, and the 1x1 LLR head.
//
// Output channel ownership: within o-tile `ot`, MFMA row r = 4g + i (g = lane/16)
// holds channel g*4*NOT + 4*ot + i, so every lane owns 4*NOT consecutive channels of
// one RE and stores them with wide vector writes. The host packs filters with the
// same permutation.
#pragma once
#include "conet_common.h"
#include "conet_kernels.h"

namespace conet {

// ---------------------------------------------------------------- vector IO helpers
template <class T>
__device__ __forceinline__ void load_vals(const T* p, float* v, int n) {
  // n consecutive elements (n * sizeof(T) is a multiple of 8 bytes, 8-byte aligned)
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int i = 0; i < n; i += 4) {
      float4 q = *reinterpret_cast<const float4*>(p + i);
      v[i] = q.x; v[i + 1] = q.y; v[i + 2] = q.z; v[i + 3] = q.w;
    }
  } else if constexpr (sizeof(T) == 2) {
#pragma unroll
    for (int i = 0; i < n; i += 4) {
      uint2 q = *reinterpret_cast<const uint2*>(p + i);
      const __bf16* b = reinterpret_cast<const __bf16*>(&q);
      v[i] = (float)b[0]; v[i + 1] = (float)b[1]; v[i + 2] = (float)b[2]; v[i + 3] = (float)b[3];
    }
  } else {
    static_assert(sizeof(T) == 8, "unsupported");
#pragma unroll
    for (int i = 0; i < n; ++i) v[i] = (float)p[i];
  }
}

__device__ __forceinline__ void load_vals(const double* p, double* v, int n) {
#pragma unroll
  for (int i = 0; i < n; ++i) v[i] = p[i];
}

template <class T, class V>
__device__ __forceinline__ void store_vals(T* p, const V* v, int n, float qscale) {
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int i = 0; i < n; i += 4)
      *reinterpret_cast<float4*>(p + i) = make_float4((float)v[i], (float)v[i + 1], (float)v[i + 2], (float)v[i + 3]);
  } else if constexpr (sizeof(T) == 8) {
#pragma unroll
    for (int i = 0; i < n; ++i) p[i] = (double)v[i];
  } else if constexpr (sizeof(T) == 2) {
#pragma unroll
    for (int i = 0; i < n; i += 4) {
      __bf16 b[4] = {f2bf((float)v[i]), f2bf((float)v[i + 1]), f2bf((float)v[i + 2]), f2bf((float)v[i + 3])};
      *reinterpret_cast<uint2*>(p + i) = *reinterpret_cast<const uint2*>(b);
    }
  } else {  // fp8, quantised with qscale = 1 / s_a of the consuming conv
#pragma unroll
    for (int i = 0; i < n; i += 8) {
      uint2 w;
      w.x = pack4_e4m3((float)v[i] * qscale, (float)v[i + 1] * qscale, (float)v[i + 2] * qscale, (float)v[i + 3] * qscale);
      w.y = pack4_e4m3((float)v[i + 4] * qscale, (float)v[i + 5] * qscale, (float)v[i + 6] * qscale, (float)v[i + 7] * qscale);
      *reinterpret_cast<uint2*>(p + i) = w;
    }
  }
}

// ---------------------------------------------------------------- tile mapping
__device__ __forceinline__ TileDesc tile_of(const ConvArgs& a, int bid) {
  if (a.tiles) return a.tiles[bid];
  TileDesc d;
  const int b = bid / a.tiles_per_slot;
  d.re_base = (int64_t)b * a.T * a.F;
  d.F = a.F;
  d.f0 = (bid - b * a.tiles_per_slot) * a.tw;
  return d;
}

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a contiguous run of
// tiles so neighbouring tiles (which share halo columns) hit the same L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  if ((nb & 7) != 0) return bid;
  return (bid & 7) * (nb >> 3) + (bid >> 3);
}

// ---------------------------------------------------------------- staging
// Stage the (TROWS) x (TW+2) halo tile of `in` (CIN channels of InT per RE) into LDS
// as Op with row pitch PITCH bytes, applying prologue and quantisation.
template <class A, class InT, int CIN, int TW, int PITCH, int NT>
__device__ __forceinline__ void stage_tile(uint8_t* lds, const InT* __restrict__ in, const TileDesc& td, int T,
                                           int prologue, const float* __restrict__ ps, const float* __restrict__ po,
                                           float qscale) {
  using Op = typename A::Op;
  constexpr int EPC = 16 / sizeof(InT) < 4 ? 4 : 16 / sizeof(InT);  // elements per global chunk
  constexpr int CPP = CIN / EPC;                                       // chunks per position
  constexpr int NPOS = TROWS * (TW + 2);
  static_assert(CIN % EPC == 0, "channel count must fill whole 16-byte chunks");
  for (int idx = threadIdx.x; idx < NPOS * CPP; idx += NT) {
    const int pos = idx / CPP, cc = idx - pos * CPP;
    const int r = pos / (TW + 2), c = pos - r * (TW + 2);
    const int t = r - 1, f = td.f0 + c - 1;
    const int ch = cc * EPC;
    float v[EPC];
    if (t >= 0 && t < T && f >= 0 && f < td.F) {
      const InT* src = in + (td.re_base + (int64_t)t * td.F + f) * CIN + ch;
      if constexpr (std::is_same<InT, Op>::value && sizeof(InT) <= 4) {  // stored as the operand: copy
        if (prologue == 0) {
          *reinterpret_cast<i32x4*>(lds + r * (TW + 2) * PITCH + c * PITCH + ch * sizeof(Op)) =
              *reinterpret_cast<const i32x4*>(src);
          continue;
        }
      }
      if constexpr (sizeof(InT) == 1) {  // fp8 operand stored by the producer: copy bytes
        *reinterpret_cast<i32x4*>(lds + r * (TW + 2) * PITCH + c * PITCH + ch) = *reinterpret_cast<const i32x4*>(src);
        continue;
      } else if constexpr (sizeof(InT) == 8) {
#pragma unroll
        for (int i = 0; i < EPC; ++i) v[i] = 0.f;
        double dv[EPC];
#pragma unroll
        for (int i = 0; i < EPC; ++i) dv[i] = (double)src[i];
        if (prologue) {
#pragma unroll
          for (int i = 0; i < EPC; ++i) {
            double z = prologue == 1 ? (double)ps[ch + i] * dv[i] + (double)po[ch + i] : dv[i];
            dv[i] = z > 0.0 ? z : 0.0;
          }
        }
        Op* dst = reinterpret_cast<Op*>(lds + r * (TW + 2) * PITCH + c * PITCH) + ch;
#pragma unroll
        for (int i = 0; i < EPC; ++i) dst[i] = (Op)dv[i];
        continue;
      } else {
        load_vals(src, v, EPC);
        if (prologue == 1) {
#pragma unroll
          for (int i = 0; i < EPC; ++i) v[i] = fmaxf(ps[ch + i] * v[i] + po[ch + i], 0.f);
        } else if (prologue == 2) {
#pragma unroll
          for (int i = 0; i < EPC; ++i) v[i] = fmaxf(v[i], 0.f);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < EPC; ++i) v[i] = 0.f;
    }
    uint8_t* dst = lds + r * (TW + 2) * PITCH + c * PITCH + ch * sizeof(Op);
    if constexpr (sizeof(Op) == 1) {
      static_assert(EPC % 4 == 0, "");
#pragma unroll
      for (int i = 0; i < EPC; i += 4)
        *reinterpret_cast<uint32_t*>(dst + i) = pack4_e4m3(v[i] * qscale, v[i + 1] * qscale, v[i + 2] * qscale, v[i + 3] * qscale);
    } else if constexpr (sizeof(Op) == 2) {
#pragma unroll
      for (int i = 0; i < EPC; i += 4) {
        __bf16 b[4] = {f2bf(v[i]), f2bf(v[i + 1]), f2bf(v[i + 2]), f2bf(v[i + 3])};
        *reinterpret_cast<uint2*>(dst + 2 * i) = *reinterpret_cast<const uint2*>(b);
      }
    } else if constexpr (sizeof(Op) == 4) {
#pragma unroll
      for (int i = 0; i < EPC; i += 4)
        *reinterpret_cast<float4*>(dst + 4 * i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
    } else {
#pragma unroll
      for (int i = 0; i < EPC; ++i) reinterpret_cast<double*>(dst)[i] = (double)v[i];
    }
  }
}

// ---------------------------------------------------------------- GEMM core
// acc[mt][ot] += W (o-tile ot) x X^T (M-tile mt) over all K steps. M-tile mt of this
// wave is global M-tile index wave + NW*mt: OFDM symbol t = idx / (TW/16), subcarrier
// block cb = idx % (TW/16).
template <class A, int CIN, int COUT, int TW, int PITCH, int NW>
struct Gemm {
  static constexpr int NOT = COUT / 16;
  static constexpr int CPT = CIN / A::VEC;                       // chunks per tap
  static constexpr int NCH = 9 * CPT;                            // real chunks
  static constexpr int CPS = 4 * A::CPL;                         // chunks per K step
  static constexpr int NS = (NCH + CPS - 1) / CPS;               // K steps
  static constexpr int MTOT = TMAX * (TW / 16);                  // M-tiles per tile (T = 14)
  static constexpr int MT = (MTOT + NW - 1) / NW;                // M-tiles per wave
  static_assert(COUT % 16 == 0, "output channels must be a multiple of 16");
  static_assert(CIN % A::VEC == 0, "");

  using AccV = typename A::AccV;

  __device__ __forceinline__ static void run(AccV (&acc)[MT][NOT], const uint8_t* lds, const i32x4* __restrict__ wp,
                                             int T, int wave, int lane) {
    const int g = lane >> 4, col = lane & 15;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ot = 0; ot < NOT; ++ot) acc[mt][ot] = AccV{};
    // base LDS byte offset of each of this wave's M-tiles for tap (0,0) (top-left)
    int base[MT];
    bool live[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int idx = wave + NW * mt;
      const int t = idx / (TW / 16), cb = idx - t * (TW / 16);
      live[mt] = (idx < MTOT) && (t < T);
      base[mt] = (t * (TW + 2) + cb * 16 + col) * PITCH;
    }
#pragma unroll 2
    for (int s = 0; s < NS; ++s) {
      i32x4 af[NOT][A::CPL];
#pragma unroll
      for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
        for (int c = 0; c < A::CPL; ++c) af[ot][c] = wp[((s * NOT + ot) * A::CPL + c) * 64 + lane];
      int off[A::CPL];
#pragma unroll
      for (int c = 0; c < A::CPL; ++c) {
        int ch = (s * 4 + g) * A::CPL + c;
        if (ch >= NCH) ch = 4 * CPT;  // padding chunk: any in-tile address (weights are 0)
        const int tap = ch / CPT, c0 = (ch - tap * CPT) * A::VEC;
        off[c] = ((tap / 3) * (TW + 2) + (tap % 3)) * PITCH + c0 * (int)sizeof(typename A::Op);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        if (!live[mt]) continue;
        i32x4 bf[A::CPL];
#pragma unroll
        for (int c = 0; c < A::CPL; ++c) bf[c] = *reinterpret_cast<const i32x4*>(lds + base[mt] + off[c]);
#pragma unroll
        for (int ot = 0; ot < NOT; ++ot) acc[mt][ot] = A::mma(af[ot], bf, acc[mt][ot]);
      }
    }
  }
};

template <class A, int CIN>
constexpr int lds_pitch() {
  int p = CIN * (int)sizeof(typename A::Op);
  return ((p / 16) % 2 == 0) ? p + 16 : p;
}

// 32 subcarriers per tile unless the halo tile would not leave room for two
// work-groups per CU, or the per-lane register budget of wide channel counts.
template <class A, int CIN, int COUT>
constexpr int tile_w() {
  return (COUT > 64 || TROWS * 34 * lds_pitch<A, CIN>() > 80 * 1024) ? 16 : 32;
}

// ---------------------------------------------------------------- the kernel
// MODE: 0 input layer, 1 first conv of a block, 2 second conv (+ residual) per branch,
// 3 second conv of all branches + product fusion + LayerNorm (+ head).
template <class A, int MODE, int CIN, int COUT, int TW, int NW>
__global__ void __launch_bounds__(NW * 64) conv3x3_kernel(ConvArgs args) {
  using Op = typename A::Op;
  using Acc = typename A::Acc;
  using AccV = typename A::AccV;
  using Act = typename A::Act;
  using Hid = typename A::Hid;
  using InT = typename std::conditional<MODE == 0, float, typename std::conditional<MODE == 1, Act, Hid>::type>::type;
  constexpr int PITCH = lds_pitch<A, CIN>();
  constexpr int NT = NW * 64;
  using G = Gemm<A, CIN, COUT, TW, PITCH, NW>;
  constexpr int MT = G::MT, NOT = G::NOT, EPL = 4 * NOT;  // EPL: channels per lane
  static_assert(sizeof(Hid) != 1 || EPL % 8 == 0, "FP8 stores write 8 channels at a time");
  __shared__ __attribute__((aligned(16))) uint8_t lds[TROWS * (TW + 2) * PITCH];

  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const TileDesc td = tile_of(args, bid);
  const int T = args.T;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  const int c0 = g * EPL;  // first channel owned by this lane

  // (t, f) of this lane's RE in each M-tile
  auto re_of = [&](int mt, int& t, int& f) {
    const int idx = wave + NW * mt;
    t = idx / (TW / 16);
    f = td.f0 + (idx - t * (TW / 16)) * 16 + col;
  };

  if constexpr (MODE != 3) {
    const int k = blockIdx.y;
    const InT* in = reinterpret_cast<const InT*>(args.in[k]);
    int prologue = 0;
    if (MODE == 1) prologue = args.pre_s[k] ? 1 : 2;
    stage_tile<A, InT, CIN, TW, PITCH, NT>(lds, in, td, T, prologue, args.pre_s[k], args.pre_o[k], args.in_qscale[k]);
    __syncthreads();
    AccV acc[MT][NOT];
    G::run(acc, lds, reinterpret_cast<const i32x4*>(args.wpack[k]), T, wave, lane);

    const float* bias = args.bias[k];
    const float* ws = args.wscale[k];
    const float deq = args.deq[k];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      int t, f;
      re_of(mt, t, f);
      if (wave + NW * mt >= G::MTOT || t >= T || f >= td.F) continue;
      const int64_t re = td.re_base + (int64_t)t * td.F + f;
      Acc v[EPL];
#pragma unroll
      for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int ch = c0 + 4 * ot + i;
          Acc a = acc[mt][ot][i];
          if constexpr (A::QUANT) a = a * (Acc)(deq * ws[ch]);
          v[4 * ot + i] = a + (Acc)bias[ch];
        }
      if constexpr (MODE == 0) {
#pragma unroll
        for (int i = 0; i < EPL; ++i) v[i] = v[i] > (Acc)0 ? v[i] : (Acc)0;
        store_vals(reinterpret_cast<Act*>(args.out[k]) + re * COUT + c0, v, EPL, 1.f);
      } else if constexpr (MODE == 1) {
        const float* s1 = args.post_s[k];
        const float* o1 = args.post_o[k];
#pragma unroll
        for (int i = 0; i < EPL; ++i) {
          Acc z = (Acc)s1[c0 + i] * v[i] + (Acc)o1[c0 + i];
          v[i] = z > (Acc)0 ? z : (Acc)0;
        }
        if (args.amax) {  // calibration: record max |h| of this branch instead of storing
          Acc mx = 0;
#pragma unroll
          for (int i = 0; i < EPL; ++i) mx = v[i] > mx ? v[i] : mx;
          atomicMax(args.amax + k, __float_as_uint((float)mx));
        } else {
          store_vals(reinterpret_cast<Hid*>(args.out[k]) + re * COUT + c0, v, EPL, args.out_qscale[k]);
        }
      } else {  // MODE 2: residual add; branch 0 of the last block feeds the head
        Acc x[EPL];
        load_vals(reinterpret_cast<const Act*>(args.resid[k]) + re * COUT + c0, x, EPL);
#pragma unroll
        for (int i = 0; i < EPL; ++i) v[i] += x[i];
        if (args.llr && k == 0) {
          Acc part[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            part[j] = 0;
            if (j < args.m)
#pragma unroll
              for (int i = 0; i < EPL; ++i) part[j] += (Acc)args.Wh[j * COUT + c0 + i] * v[i];
          }
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            part[j] += __shfl_xor(part[j], 16);
            part[j] += __shfl_xor(part[j], 32);
          }
#pragma unroll
          for (int j = 0; j < 8; ++j)
            if (j < args.m && (j & 3) == g) args.llr[re * args.m + j] = (float)(part[j] + (Acc)args.bh[j]);
        } else if (args.out[k]) {
          store_vals(reinterpret_cast<Act*>(args.out[k]) + re * COUT + c0, v, EPL, 1.f);
        }
      }
    }
  } else {
    // ---- all K branches of the second conv in this work-group, product held in registers
    Acc P[MT][EPL];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int i = 0; i < EPL; ++i) P[mt][i] = (Acc)1;
    for (int k = 0; k < args.K; ++k) {
      if (k) __syncthreads();  // LDS reuse
      stage_tile<A, InT, CIN, TW, PITCH, NT>(lds, reinterpret_cast<const InT*>(args.in[k]), td, T, 0, nullptr,
                                             nullptr, args.in_qscale[k]);
      __syncthreads();
      AccV acc[MT][NOT];
      G::run(acc, lds, reinterpret_cast<const i32x4*>(args.wpack[k]), T, wave, lane);
      const float* bias = args.bias[k];
      const float* ws = args.wscale[k];
      const float deq = args.deq[k];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        int t, f;
        re_of(mt, t, f);
        if (wave + NW * mt >= G::MTOT || t >= T || f >= td.F) continue;
        const int64_t re = td.re_base + (int64_t)t * td.F + f;
        Acc x[EPL], v[EPL];
        load_vals(reinterpret_cast<const Act*>(args.resid[k]) + re * COUT + c0, x, EPL);
#pragma unroll
        for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int ch = c0 + 4 * ot + i;
            Acc a = acc[mt][ot][i];
            if constexpr (A::QUANT) a = a * (Acc)(deq * ws[ch]);
            v[4 * ot + i] = x[4 * ot + i] + a + (Acc)bias[ch];
          }
        if (args.out[k] && k > 0) store_vals(reinterpret_cast<Act*>(args.out[k]) + re * COUT + c0, v, EPL, 1.f);
        if (args.save_o[k]) store_vals(reinterpret_cast<Act*>(args.save_o[k]) + re * COUT + c0, v, EPL, 1.f);
#pragma unroll
        for (int i = 0; i < EPL; ++i) P[mt][i] *= v[i];
      }
    }
    // ---- per-RE LayerNorm over the C channels (4 lanes x EPL channels)
    const Acc invC = (Acc)1 / (Acc)COUT;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      int t, f;
      re_of(mt, t, f);
      if (wave + NW * mt >= G::MTOT || t >= T || f >= td.F) continue;
      const int64_t re = td.re_base + (int64_t)t * td.F + f;
      Acc s = 0;
#pragma unroll
      for (int i = 0; i < EPL; ++i) s += P[mt][i];
      s += __shfl_xor(s, 16);
      s += __shfl_xor(s, 32);
      const Acc mu = s * invC;
      Acc q = 0;
#pragma unroll
      for (int i = 0; i < EPL; ++i) { const Acc d = P[mt][i] - mu; q += d * d; }
      q += __shfl_xor(q, 16);
      q += __shfl_xor(q, 32);
      Acc rs;
      if constexpr (sizeof(Acc) == 8) rs = (Acc)1 / sqrt(q * invC + (Acc)args.eps);
      else rs = (Acc)1 / sqrtf(q * invC + (Acc)args.eps);
      Acc v[EPL];
#pragma unroll
      for (int i = 0; i < EPL; ++i) v[i] = (Acc)args.gamma[c0 + i] * (P[mt][i] - mu) * rs + (Acc)args.beta[c0 + i];
      if (args.llr) {
        Acc part[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          part[j] = 0;
          if (j < args.m)
#pragma unroll
            for (int i = 0; i < EPL; ++i) part[j] += (Acc)args.Wh[j * COUT + c0 + i] * v[i];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          part[j] += __shfl_xor(part[j], 16);
          part[j] += __shfl_xor(part[j], 32);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < args.m && (j & 3) == g) args.llr[re * args.m + j] = (float)(part[j] + (Acc)args.bh[j]);
      }
      if (args.out[0]) store_vals(reinterpret_cast<Act*>(args.out[0]) + re * COUT + c0, v, EPL, 1.f);
    }
  }
}

// ---------------------------------------------------------------- launch
template <class A, int MODE, int CIN, int COUT>
static hipError_t launch_one(ConvArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  constexpr int TW = tile_w<A, CIN, COUT>();
  a.tw = TW;
  hipLaunchKernelGGL((conv3x3_kernel<A, MODE, CIN, COUT, TW, CONV_NW>), dim3(n_tiles, grid_y), dim3(CONV_NW * 64), 0,
                     s, a);
  return hipGetLastError();
}

template <class A, int CIN, int COUT>
static hipError_t launch_mode(int mode, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  switch (mode) {
    case 0: return launch_one<A, 0, CIN, COUT>(a, n_tiles, grid_y, s);
    case 1: return launch_one<A, 1, CIN, COUT>(a, n_tiles, grid_y, s);
    case 2: return launch_one<A, 2, CIN, COUT>(a, n_tiles, grid_y, s);
    case 3: return launch_one<A, 3, CIN, COUT>(a, n_tiles, grid_y, s);
  }
  return hipErrorInvalidValue;
}

// Channel pairs instantiated: input layers (C_in -> C) and blocks (C -> C) of the
// workloads (C_in 8/16/32, C 16/32/64/96).
#define CONET_PAIRS(X) X(8, 16) X(8, 32) X(8, 64) X(16, 16) X(16, 32) X(16, 64) X(32, 32) X(32, 96) X(64, 64) X(96, 96)
#define CONET_PAIRS_FP8(X) X(16, 32) X(16, 64) X(32, 32) X(32, 64) X(32, 96) X(64, 64) X(96, 96)

template <class A>
hipError_t launch_dtype(int mode, int cin, int cout, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s) {
#define CONET_CASE(CI, CO) \
  if (cin == CI && cout == CO) return launch_mode<A, CI, CO>(mode, a, n_tiles, grid_y, s);
  if constexpr (sizeof(typename A::Op) == 1) {
    CONET_PAIRS_FP8(CONET_CASE)
  } else {
    CONET_PAIRS(CONET_CASE)
  }
#undef CONET_CASE
  return hipErrorInvalidValue;
}

template <class A>
int tile_width_dtype(int cin, int cout) {
#define CONET_TW(CI, CO) \
  if (cin == CI && cout == CO) return tile_w<A, CI, CO>();
  if constexpr (sizeof(typename A::Op) == 1) {
    CONET_PAIRS_FP8(CONET_TW)
  } else {
    CONET_PAIRS(CONET_TW)
  }
#undef CONET_TW
  return 0;
}

}  // namespace conet
