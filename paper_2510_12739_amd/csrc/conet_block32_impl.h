// Fused residual block of the CoNet-Rx forward pass at 96 channels (gfx950) on the 32x32
// MFMAs: v_mfma_f32_32x32x64_f8f6f4 (FP8) and v_mfma_f32_32x32x16_bf16 (BF16).
//
// The dataflow is that of the fused block kernel (conet_block_impl.h): stage pre(x) with
// a two-RE halo, conv 1 over the (14 x TWO+2) region, h into LDS in place of x, conv 2
// over the 14 x TWO output region and the block output (residual, fusion, LayerNorm,
// head). Only the implicit GEMMs differ: one instruction covers 32 output channels x 32
// REs x 64 (FP8) or 16 (BF16) input taps. At 96 channels the 16x16 tilings need six
// accumulator tiles and six filter fragments per K step per lane, which leaves no
// registers for a prefetch ring (the FP8 kernel spills); the 32x32 tiling needs half the
// filter registers for the same REs per wave and reads half the LDS bytes per MFMA.
//
// Operand layouts (lane l, r = l % 32, h = l / 32). A 16-byte chunk holds 16 (FP8) or 8
// (BF16) channels; a lane supplies CPL = 2 (FP8) or 1 (BF16) chunks per instruction. Each
// lane half walks its own half of the channels: half h takes, per tap, the HC chunks of
// channels 48h .. 48h+47 (HC = 3 or 6), in the sequence u = 0 .. 9 HC - 1 (tap u / HC,
// chunk HC h + u % HC), CPL per K step (past the end: zero padding). So half 1 always
// reads 48 channels after half 0, an offset folded into the lane's base address.
//   filter (A): row r of output tile ot, the chunks of half h in step s;
//   activations (B): RE r of the M-tile, the same chunks;
//   accumulator: register i holds row 8(i/4) + 4h + i%4 of RE r.
// Filter rows are packed (pack_filter32) so that lane half h holds the 48 contiguous
// channels 48h .. 48h+47 of its RE: register i of tile ot is channel 48h + 16 ot + i.
#pragma once
#include "conet_block_impl.h"

namespace conet {

constexpr int B32_C = 96;

__device__ __forceinline__ i32x8 cat8(const i32x4* x) {
  return __builtin_shufflevector(x[0], x[1], 0, 1, 2, 3, 4, 5, 6, 7);
}

// The two operand formats. C: channels (a multiple of 32); CPL: 16-byte chunks per lane per
// instruction; CHC: channels per chunk; TWO: output subcarriers per tile (the x tile of
// 16 x (TWO + 4) positions leaves room for two work-groups per CU); ADEPTH: filter prefetch
// distance in K steps (registers).
struct Mfma32FP8 {
  using A = ArithFP8;
  static constexpr int C = B32_C, CPL = 2, CHC = 16, TWO = 22, ADEPTH = 2;
  __device__ __forceinline__ static f32x16 mma(const i32x4* a, const i32x4* b, f32x16 c) {
    return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(cat8(a), cat8(b), c, 0, 0, 0, 0, 0, 0);
  }
};
template <int C_ = B32_C>
struct Mfma32BF16 {
  using A = ArithBF16;
  static constexpr int C = C_, CPL = 1, CHC = 8, TWO = C_ == 96 ? 18 : 30, ADEPTH = 2;
  __device__ __forceinline__ static f32x16 mma(const i32x4* a, const i32x4* b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a[0]), __builtin_bit_cast(bf16x8, b[0]), c,
                                                   0, 0, 0);
  }
};

// One wave's implicit GEMM over MT M-tiles of 32 REs (LDS byte offsets base[mt] of the
// tap (-1, -1) operand of each lane's RE) and all 96 output channels.
template <class M, int ROWP, int PITCH, int MT>
struct GemmCore32 {
  static constexpr int C = M::C, NOT = C / 32, CPL = M::CPL, HC = C / 2 / M::CHC, NU = 9 * HC;
  static constexpr int NS = (NU + CPL - 1) / CPL, ADEPTH = M::ADEPTH, NA = ADEPTH + 1;
  static constexpr int HALF = 16 * HC;  // byte offset of lane half 1's chunks

  // LDS byte offset of chunk c of lane half 0 in K step s
  __device__ __forceinline__ static constexpr int b_off(int s, int c) {
    int u = CPL * s + c;
    if (u >= NU) u = 0;  // padding chunk: any in-tile address (its weights are 0)
    const int tap = u / HC;
    return ((tap / 3) * ROWP + (tap % 3)) * PITCH + (u - tap * HC) * 16;
  }

  __device__ __forceinline__ static void load_a(i32x4 (&a)[NOT][CPL], const i32x4* __restrict__ wp, int s,
                                                int lane) {
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int c = 0; c < CPL; ++c) a[ot][c] = wp[((s * NOT + ot) * 64 + lane) * CPL + c];
  }

  __device__ __forceinline__ static void load_b(i32x4 (&b)[CPL], const uint8_t* lds, int base, int s) {
#pragma unroll
    for (int c = 0; c < CPL; ++c) b[c] = *reinterpret_cast<const i32x4*>(lds + base + b_off(s, c));
  }

  // Filter fragments are prefetched ADEPTH steps ahead; activation fragments alternate
  // between two buffers, the next (step, M-tile)'s read issued before this one's MFMAs (its
  // LDS latency hides behind three MFMAs), which leaves the registers for the filter ring.
  // base[mt]: LDS byte offset of the lane's RE at tap (-1, -1), lane half included.
  __device__ __forceinline__ static void run(f32x16 (&acc)[MT][NOT], const uint8_t* lds, const i32x4* __restrict__ wp,
                                             const int (&base)[MT], int lane) {
    __builtin_amdgcn_s_setprio(1);  // the MFMA loop issues ahead of the other work-group's waves
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ot = 0; ot < NOT; ++ot) acc[mt][ot] = f32x16{};
    i32x4 a[NA][NOT][CPL];
    i32x4 b[2][CPL];  // ping-pong: the fragment of the next (step, M-tile) is read before this one's MFMAs
#pragma unroll
    for (int d = 0; d < ADEPTH; ++d) load_a(a[d], wp, d, lane);
    load_b(b[0], lds, base[0], 0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (s + ADEPTH < NS) load_a(a[(s + ADEPTH) % NA], wp, s + ADEPTH, lane);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int i = s * MT + mt;
        if (mt + 1 < MT) load_b(b[(i + 1) & 1], lds, base[mt + 1], s);
        else if (s + 1 < NS) load_b(b[(i + 1) & 1], lds, base[0], s + 1);
#pragma unroll
        for (int ot = 0; ot < NOT; ++ot) acc[mt][ot] = M::mma(a[s % NA][ot], b[i & 1], acc[mt][ot]);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    __builtin_amdgcn_s_setprio(0);
  }
};

template <class M>
constexpr int block32_lds_bytes() {
  return TROWS * (M::TWO + 4) * lds_pitch<typename M::A, M::C>() + NPAR * M::C * 4;
}

// One fused residual block of branch k on tile `bid` (before the XCD remap); MAIN, HEAD and
// NSUP as in block_body.
template <class M, bool MAIN, bool HEAD, int NSUP>
__device__ __forceinline__ void block32_body(const BlockArgs& args, int k, uint8_t* lds) {
  using A = typename M::A;
  using Act = typename A::Act;
  constexpr int TWO = M::TWO;
  constexpr int C = M::C, NW = CONV_NW, NT = NW * 64;
  constexpr int XW = TWO + 4, HW = TWO + 2;  // LDS positions per row: x tile, h tile
  constexpr int PITCH = lds_pitch<A, C>();
  constexpr int Q1 = TMAX * HW, Q2 = TMAX * TWO;  // REs of the conv-1 and conv-2 regions
  constexpr int M1 = (Q1 + 31) / 32, M2 = (Q2 + 31) / 32;
  constexpr int MT1 = (M1 + NW - 1) / NW, MT2 = (M2 + NW - 1) / NW;
  constexpr int NOT = C / 32, EPL = C / 2;
  constexpr int TILE = TROWS * XW * PITCH;
  using G1 = GemmCore32<M, XW, PITCH, MT1>;
  using G2 = GemmCore32<M, HW, PITCH, MT2>;
  static_assert(2 * (TILE + NPAR * C * 4) <= 160 * 1024, "LDS must leave room for two work-groups per CU");
  static_assert(PITCH % 16 == 0 && EPL % 16 == 0, "h rows are written in 16-byte chunks");
  float* par = reinterpret_cast<float*>(lds + TILE);

  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const TileDesc td = tile_of(args, bid);
  const int T = args.T;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int h = lane >> 5, col = lane & 31;
  const int c0 = h * EPL;  // first channel owned by this lane

  // 0. per-channel parameters: loads issued now, written to LDS after the tile's loads
  constexpr int NPV = (NPAR * C + NT - 1) / NT;
  float pv[NPV];
#pragma unroll
  for (int u = 0; u < NPV; ++u) {
    const int i = threadIdx.x + u * NT;
    const int pi = i / C, c = i - pi * C;
    float val = 0.f;
    switch (pi) {
      case P_B1: val = args.b1[k][c]; break;
      case P_S1: val = args.post_s[k][c]; break;
      case P_O1: val = args.post_o[k][c]; break;
      case P_Q1: val = A::QUANT ? args.deq1[k] * args.ws1[k][c] : 1.f; break;
      case P_B2: val = args.b2[k][c]; break;
      case P_Q2: val = A::QUANT ? args.deq2[k] * args.ws2[k][c] : 1.f; break;
      case P_GAM: val = MAIN ? args.gamma[c] : 0.f; break;
      case P_BET: val = MAIN ? args.beta[c] : 0.f; break;
      default: break;
    }
    pv[u] = val;
  }

  // 1. pre(x) with a two-RE halo; LDS row r = symbol r - 1, column c = subcarrier f0 + c - 2
  stage_tile<A, Act, C, XW, 2, PITCH, NT>(lds, reinterpret_cast<const Act*>(args.x[k]), td, T,
                                          args.pre_s[k] ? 1 : 2, args.pre_s[k], args.pre_o[k], args.q1[k]);
#pragma unroll
  for (int u = 0; u < NPV; ++u)
    if (threadIdx.x + u * NT < NPAR * C) par[threadIdx.x + u * NT] = pv[u];
  __syncthreads();

  // 2. conv 1 on RE q = t * HW + j of the region (symbol t, subcarrier f0 - 1 + j)
  f32x16 acc1[MT1][NOT];
  {
    int base[MT1];
#pragma unroll
    for (int mt = 0; mt < MT1; ++mt) {
      int q = (wave + NW * mt) * 32 + col;
      if (q >= Q1) q = Q1 - 1;  // surplus lanes recompute a real RE (never written)
      const int t = q / HW, j = q - t * HW;
      base[mt] = (t * XW + j) * PITCH + G1::HALF * h;  // tap (-1, -1): x row t (symbol t - 1), column j
    }
    G1::run(acc1, lds, reinterpret_cast<const i32x4*>(args.w1[k]), base, lane);
  }
  __syncthreads();  // every wave has read its last x operand: h may overwrite the tile

  // 3. h = ReLU(s1 (dequant(conv) + b1) + o1), zero for REs outside the slot (conv 2's
  //    zero padding), into LDS row t + 1 (symbol t), column j in the operand type (FP8 with
  //    conv 2's input scale). Four channels at a time, parameters read from LDS next to
  //    their use (held for the whole tile they would not fit the registers).
  const float qs = args.q2[k];
  (void)qs;
#pragma unroll
  for (int mt = 0; mt < MT1; ++mt) {
    const int q = (wave + NW * mt) * 32 + col;
    if (wave + NW * mt >= M1 || q >= Q1) continue;
    const int t = q / HW, j = q - t * HW;
    const int f = td.f0 - 1 + j;
    const bool valid = t < T && f >= 0 && f < td.F;
    uint8_t* dst = lds + ((t + 1) * HW + j) * PITCH + c0 * (int)sizeof(typename A::Op);
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot) {
      i32x4 w[sizeof(typename A::Op)];  // 16 channels: 16 bytes (FP8) or 32 (BF16)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = c0 + 16 * ot + 4 * u;
        const float4 pb = *reinterpret_cast<const float4*>(par + P_B1 * C + e);
        const float4 ps = *reinterpret_cast<const float4*>(par + P_S1 * C + e);
        const float4 po = *reinterpret_cast<const float4*>(par + P_O1 * C + e);
        const float4 pq = *reinterpret_cast<const float4*>(par + P_Q1 * C + e);
        const f32x16& a = acc1[mt][ot];
        // a select, not a branch: z is computed anyway
        float q0 = a[4 * u + 0], q1 = a[4 * u + 1], q2 = a[4 * u + 2], q3 = a[4 * u + 3];
        if constexpr (A::QUANT) { q0 *= pq.x; q1 *= pq.y; q2 *= pq.z; q3 *= pq.w; }
        const float h0 = fmaxf(valid ? ps.x * (q0 + pb.x) + po.x : -1.f, 0.f);
        const float h1 = fmaxf(valid ? ps.y * (q1 + pb.y) + po.y : -1.f, 0.f);
        const float h2 = fmaxf(valid ? ps.z * (q2 + pb.z) + po.z : -1.f, 0.f);
        const float h3 = fmaxf(valid ? ps.w * (q3 + pb.w) + po.w : -1.f, 0.f);
        if constexpr (A::QUANT) {
          w[0][u] = (int)pack4_e4m3(h0 * qs, h1 * qs, h2 * qs, h3 * qs);
        } else {
          const __bf16 bb[4] = {f2bf(h0), f2bf(h1), f2bf(h2), f2bf(h3)};
          const uint2 pk = *reinterpret_cast<const uint2*>(bb);
          w[u / 2][2 * (u % 2)] = (int)pk.x;
          w[u / 2][2 * (u % 2) + 1] = (int)pk.y;
        }
      }
#pragma unroll
      for (int v = 0; v < (int)sizeof(typename A::Op); ++v)
        *reinterpret_cast<i32x4*>(dst + 16 * ((int)sizeof(typename A::Op) * ot + v)) = w[v];
    }
  }
  {  // h rows of symbols -1 and 14 (rows t in [T, 14) were written as zeros above)
    constexpr int CH = C * (int)sizeof(typename A::Op) / 16;  // 16-byte chunks per position
    for (int i = threadIdx.x; i < 2 * HW * CH; i += NT) {
      const int rr = i / (HW * CH), rem = i - rr * HW * CH;
      const int j = rem / CH, ch = rem - j * CH;
      *reinterpret_cast<i32x4*>(lds + ((rr ? TROWS - 1 : 0) * HW + j) * PITCH + ch * 16) = i32x4{0, 0, 0, 0};
    }
  }
  __syncthreads();

  // 4. conv 2 on RE q = t * TWO + j of the output region (symbol t, subcarrier f0 + j)
  f32x16 acc2[MT2][NOT];
  {
    int base[MT2];
#pragma unroll
    for (int mt = 0; mt < MT2; ++mt) {
      int q = (wave + NW * mt) * 32 + col;
      if (q >= Q2) q = Q2 - 1;
      const int t = q / TWO, j = q - t * TWO;
      base[mt] = (t * HW + j) * PITCH + G2::HALF * h;  // tap (-1, -1): h row t (symbol t - 1), column j
    }
    G2::run(acc2, lds, reinterpret_cast<const i32x4*>(args.w2[k]), base, lane);
  }
  const bool head = HEAD && (MAIN || k == 0);

  // 5. block output. The head weights (read by every M-tile) are copied into the now
  //    free LDS tile once.
  float* whl = reinterpret_cast<float*>(lds);
  if constexpr (HEAD) {
    __syncthreads();  // every wave has read its last h operand
    const int nwh = args.m * C;
    for (int i = threadIdx.x; i < nwh + 8; i += NT)
      whl[i] = i < nwh ? args.Wh[i] : (i - nwh < args.m ? args.bh[i - nwh] : 0.f);
    __syncthreads();
  }
  constexpr int NR = EPL * (int)sizeof(Act) / 16;  // 16-byte vectors of one lane's activations
  auto load_act = [&](const void* src, int64_t re, float* v) {
    const i32x4* p = reinterpret_cast<const i32x4*>(reinterpret_cast<const Act*>(src) + re * C + c0);
    i32x4 raw[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) raw[r] = p[r];
    unpack_raw<Act, i32x4, EPL>(raw, v);
  };
#pragma unroll
  for (int mt = 0; mt < MT2; ++mt) {
    const int q = (wave + NW * mt) * 32 + col;
    const int t = q / TWO, j = q - t * TWO;
    const int f = td.f0 + j;
    if (wave + NW * mt >= M2 || q >= Q2 || t >= T || f >= td.F) continue;
    const int64_t re = td.re_base + (int64_t)t * td.F + f;
    float v[EPL];
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int i = 0; i < 16; i += 4) {
        const float4 pb = *reinterpret_cast<const float4*>(par + P_B2 * C + c0 + 16 * ot + i);
        float4 pq = make_float4(1.f, 1.f, 1.f, 1.f);
        if constexpr (A::QUANT) pq = *reinterpret_cast<const float4*>(par + P_Q2 * C + c0 + 16 * ot + i);
        v[16 * ot + i + 0] = acc2[mt][ot][i + 0] * pq.x + pb.x;
        v[16 * ot + i + 1] = acc2[mt][ot][i + 1] * pq.y + pb.y;
        v[16 * ot + i + 2] = acc2[mt][ot][i + 2] * pq.z + pb.z;
        v[16 * ot + i + 3] = acc2[mt][ot][i + 3] * pq.w + pb.w;
        __builtin_amdgcn_sched_barrier(0);
      }
    auto x_fn = [&](float* x) { load_act(args.x[k], re, x); };
    auto sup_fn = [&](int kk, float* sv) { load_act(args.sup[kk], re, sv); };
    finish_block<A, C, EPL, NSUP, decltype(x_fn), decltype(sup_fn), 2>(
        v, re, c0, h, MAIN, x_fn, sup_fn, MAIN ? args.out[0] : args.out[k], (MAIN || k == 0) ? args.save_o0 : nullptr,
        head, NSUP + 1, par + P_GAM * C, par + P_BET * C, args.eps, whl, whl + args.m * C, args.llr, args.m,
        args.fusion_sum != 0, (MAIN && args.feedback) ? const_cast<void* const*>(args.sup) : nullptr,
        args.norm_affine != 0);
  }
}

template <class M, bool MAIN, bool HEAD, int NSUP>
__global__ void __launch_bounds__(CONV_NW * 64, 2) block32_kernel(BlockArgs args) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[block32_lds_bytes<M>()];
  block32_body<M, MAIN, HEAD, NSUP>(args, blockIdx.y + args.k_off, lds);
}

// Main branch of block l (blockIdx.y == 0) with the support branches of block l + 1, as
// block_pair_kernel.
template <class M, int NSUP>
__global__ void __launch_bounds__(CONV_NW * 64, 2) block32_pair_kernel(BlockArgs args) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[block32_lds_bytes<M>()];
  if (blockIdx.y == 0)
    block32_body<M, true, false, NSUP>(args, 0, lds);
  else
    block32_body<M, false, false, 0>(args, blockIdx.y, lds);
}

template <class M, bool HEAD>
static hipError_t launch_block32_h(int kind, BlockArgs& a, dim3 grid, hipStream_t s) {
  const dim3 blk(CONV_NW * 64);
  if (kind == BLOCK_PLAIN) {
    hipLaunchKernelGGL((block32_kernel<M, false, HEAD, 0>), grid, blk, 0, s, a);
  } else if (kind == BLOCK_MAIN) {
    switch (a.K) {
      case 1: hipLaunchKernelGGL((block32_kernel<M, true, HEAD, 0>), grid, blk, 0, s, a); break;
      case 2: hipLaunchKernelGGL((block32_kernel<M, true, HEAD, 1>), grid, blk, 0, s, a); break;
      case 3: hipLaunchKernelGGL((block32_kernel<M, true, HEAD, 2>), grid, blk, 0, s, a); break;
      case 4: hipLaunchKernelGGL((block32_kernel<M, true, HEAD, 3>), grid, blk, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {  // BLOCK_PAIR: no head
    if constexpr (HEAD) return hipErrorInvalidValue;
    switch (a.K) {
      case 2: hipLaunchKernelGGL((block32_pair_kernel<M, 1>), grid, blk, 0, s, a); break;
      case 3: hipLaunchKernelGGL((block32_pair_kernel<M, 2>), grid, blk, 0, s, a); break;
      case 4: hipLaunchKernelGGL((block32_pair_kernel<M, 3>), grid, blk, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

// One tile width at every batch size (18 or 22 subcarriers already give a slot 149+ tiles).
// The kernels never save h (hid_out must be null): FP8 models are inference-only and BF16
// training models at 96 channels run the two-conv path, whose filter packs the optimiser
// keeps current.
template <class M>
hipError_t launch_block32(int kind, BlockArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  for (int k = 0; k < KMAX_ARGS; ++k)
    if (a.hid_out[k]) return hipErrorInvalidValue;
  a.tw = M::TWO;
  if (a.llr && (a.m < 1 || a.m > 8)) return hipErrorInvalidValue;
  const dim3 grid(n_tiles, grid_y);
  return a.llr ? launch_block32_h<M, true>(kind, a, grid, s) : launch_block32_h<M, false>(kind, a, grid, s);
}

}  // namespace conet
