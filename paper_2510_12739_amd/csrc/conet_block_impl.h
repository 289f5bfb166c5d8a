// Fused residual block of the CoNet-Rx forward pass (gfx950): both 3x3 convs of one
// block of one branch in a single launch, with the hidden activation h kept in LDS.
//
// A block computes O = x + W2 * ReLU(s1 (W1 * pre(x) + b1) + o1) + b2 with
// pre(x) = ReLU(s0 x + o0) (ReLU(x) on the main branch after a fusion). Run as two
// convs, h makes a round trip through HBM and x is read twice; here one work-group
// owns one tile (a slot, its T <= 14 symbols, TWO output subcarriers) and:
//   1. stages pre(x) for subcarriers f0-2 .. f0+TWO+1 (two-RE halo) into LDS,
//   2. runs conv 1 on the (14 x TWO+2) region that conv 2 needs (MFMA, h in registers),
//   3. after a barrier, overwrites the x tile with h (zero outside the slot, rounded to
//      the operand type exactly as a stored h would be),
//   4. runs conv 2 on the 14 x TWO output region and finishes the block: residual add
//      and, on the main branch of a fused block, the product with the stored support
//      outputs, the LayerNorm and the LLR head.
// HBM traffic per branch drops from five activation passes (x, h written, h read, x
// read again, O written) to two plus the residual re-read, which hits L2 or the
// last-level cache. The conv-1 halo recompute costs (TWO+2)/TWO of conv 1's MFMAs.
//
// M-tiles are 16 consecutive REs of a region flattened row-major (t, j), so they may
// straddle two OFDM symbols; each lane computes its own LDS address, so the GEMM core
// does not care. Both GEMMs use the register-pipelined core of the single-conv kernel.
#pragma once
#include "conet_conv_impl.h"

namespace conet {

// Output subcarriers per fused tile (0: no fused kernel for this type / width). The
// x tile of TROWS x (TWO+4) positions must leave room for two work-groups per CU, and
// conv 1's accumulators (ceil(14 (TWO+2) / 64) M-tiles per wave) must fit the
// per-lane register budget.
// W = TW_NARROW: the tile width for batches whose wide tiles cannot fill the GPU (one slot,
// a serving batch): more, shorter work-groups cut the latency of each launch at the cost of
// halo recompute. W = TW_NARROW3 (64 channels only, 0 elsewhere): such a batch whose paired
// launches hold more narrow work-groups than two per CU; built for three per CU. The
// arithmetic per RE is the same at every width, so results are bit-identical whichever
// width a batch runs at.
template <class A, int C, int W = TW_WIDE>
constexpr int block_tw() {
  if constexpr (std::is_same<A, ArithBF16>::value) {
    if (C == 64) return W == TW_NARROW3 ? 13 : W == TW_NARROW ? 14 : 30;
    if (W == TW_NARROW3) return 0;
    return C == 32 ? 44 : C == 16 ? 60 : 0;
  }
  return 0;
}

// Work-groups per CU the fused kernel is built for (LDS tile and register budget). Three
// (18-subcarrier tiles, 168 VGPRs) measured slower than two on the C = 64 workload: more
// halo recompute and padded M-tiles, and no room left to prefetch the epilogue inputs.
// The TW_NARROW3 width is built for three: on a batch too small to fill the GPU a
// work-group's time is set by latency rather than by the CU's throughput, and three per CU
// let the paired launch of one full-band slot (3 x 252 work-groups at K = 3) run in one
// round instead of two.
template <class A, int C, int TWO>
constexpr int block_occ() {
  return TWO == block_tw<A, C, TW_NARROW3>() ? 3 : 2;
}

// Raw 16-byte (or 8-byte) vectors holding one lane's EPL activation values of one RE.
template <class Act, int EPL>
using RawOf = typename std::conditional<(EPL * sizeof(Act)) % 16 == 0, i32x4, uint2>::type;

template <class Act, class RawT, int EPL, class Acc>
__device__ __forceinline__ void unpack_raw(const RawT* r, Acc* v) {
  const Act* a = reinterpret_cast<const Act*>(r);
#pragma unroll
  for (int i = 0; i < EPL; ++i) v[i] = (Acc)(float)a[i];
}

// Per-channel parameters of a block, staged once per work-group into LDS behind the
// tile (FP32, C each): conv-1 bias, the affine after conv 1, the dequantisation factors
// of both convs (FP8; ones otherwise), conv-2 bias and the LayerNorm affine.
enum { P_B1, P_S1, P_O1, P_Q1, P_B2, P_Q2, P_GAM, P_BET, NPAR };

// LDS bytes of one work-group of the fused kernel: the x / h tile, then the parameters.
template <class A, int C, int TWO>
constexpr int block_lds_bytes() {
  return TROWS * (TWO + 4) * lds_pitch<A, C>() + NPAR * C * 4;
}

// One fused residual block of branch k on tile `bid` of the launch's tile list.
// MAIN: the main branch of a fused block (fusion epilogue); NSUP: the support branches it
// fuses (K - 1; 0 otherwise). HEAD: this block feeds the LLR head (after the last block).
template <class A, int C, int TWO, bool MAIN, bool HEAD, int NSUP>
__device__ __forceinline__ void block_body(const BlockArgs& args, int k, uint8_t* lds, int bid) {
  using Acc = typename A::Acc;
  using AccV = typename A::AccV;
  using Act = typename A::Act;
  using Op = typename A::Op;
  constexpr int NW = CONV_NW, NT = NW * 64;
  constexpr int XW = TWO + 4, HW = TWO + 2;  // LDS positions per row: x tile, h tile
  constexpr int PITCH = lds_pitch<A, C>();
  constexpr int Q1 = TMAX * HW, Q2 = TMAX * TWO;  // REs of the conv-1 and conv-2 regions
  constexpr int M1 = (Q1 + 15) / 16, M2 = (Q2 + 15) / 16;
  constexpr int MT1 = (M1 + NW - 1) / NW, MT2 = (M2 + NW - 1) / NW;
  constexpr int NOT = C / 16, EPL = 4 * NOT;
  constexpr int TILE = TROWS * XW * PITCH;
  constexpr int OCC = block_occ<A, C, TWO>();
  constexpr int VB = OCC >= 3 ? 120 : 200;  // accumulator + operand VGPRs of the GEMM loops
  using G1 = GemmCore<A, C, C, XW, PITCH, MT1, VB>;
  using G2 = GemmCore<A, C, C, HW, PITCH, MT2, VB>;
  static_assert(OCC * (TILE + NPAR * C * 4) <= 160 * 1024, "LDS must leave room for OCC work-groups per CU");
  static_assert((C * (int)sizeof(Op)) % 16 == 0, "h rows are written in 16-byte chunks");
  float* par = reinterpret_cast<float*>(lds + TILE);

  const TileDesc td = tile_of(args, bid);
  const int T = args.T;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  const int c0 = g * EPL;  // first channel owned by this lane

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
  AccV acc1[MT1][NOT];
  {
    int base[MT1];
#pragma unroll
    for (int mt = 0; mt < MT1; ++mt) {
      int q = (wave + NW * mt) * 16 + col;
      if (q >= Q1) q = Q1 - 1;  // surplus lanes recompute a real RE (never written)
      const int t = q / HW, j = q - t * HW;
      base[mt] = (t * XW + j) * PITCH;  // tap (-1, -1): x row t (symbol t - 1), column j
    }
    G1::run(acc1, lds, reinterpret_cast<const i32x4*>(args.w1[k]), base, lane);
  }
  float pb[EPL], ps[EPL], po[EPL], pq[EPL];
#pragma unroll
  for (int i = 0; i < EPL; ++i) {
    pb[i] = par[P_B1 * C + c0 + i];
    ps[i] = par[P_S1 * C + c0 + i];
    po[i] = par[P_O1 * C + c0 + i];
    pq[i] = par[P_Q1 * C + c0 + i];
  }
  __syncthreads();  // every wave has read its last x operand: h may overwrite the tile

  // 3. h = ReLU(s1 (conv + b1) + o1) into LDS row t + 1 (symbol t), column j; zero for
  //    REs outside the slot (conv 2's zero padding)
#pragma unroll
  for (int mt = 0; mt < MT1; ++mt) {
    const int q = (wave + NW * mt) * 16 + col;
    if (wave + NW * mt >= M1 || q >= Q1) continue;
    const int t = q / HW, j = q - t * HW;
    const int f = td.f0 - 1 + j;
    const bool valid = t < T && f >= 0 && f < td.F;
    float v[EPL];
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int e = 4 * ot + i;
        Acc a = acc1[mt][ot][i];
        if constexpr (A::QUANT) a = a * (Acc)pq[e];
        const float z = ps[e] * (float)(a + (Acc)pb[e]) + po[e];
        v[e] = fmaxf(valid ? z : -1.f, 0.f);  // a select, not a branch: z is computed anyway
      }
    if (args.hid_out[k] && valid && j >= 1 && j <= TWO) {  // training: h of this tile's own REs
      const int64_t re = td.re_base + (int64_t)t * td.F + f;
      store_vals(reinterpret_cast<typename A::Hid*>(args.hid_out[k]) + re * C + c0, v, EPL, args.q2[k]);
    }
    uint8_t* dst = lds + ((t + 1) * HW + j) * PITCH + c0 * (int)sizeof(Op);
    if constexpr (sizeof(Op) == 2) {
#pragma unroll
      for (int i = 0; i < EPL; i += 8) {
        __bf16 bb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) bb[u] = f2bf(v[i + u]);
        *reinterpret_cast<i32x4*>(dst + 2 * i) = *reinterpret_cast<const i32x4*>(bb);
      }
    } else if constexpr (sizeof(Op) == 1) {
      const float qs = args.q2[k];
#pragma unroll
      for (int i = 0; i < EPL; i += 8) {
        uint2 w;
        w.x = pack4_e4m3(v[i] * qs, v[i + 1] * qs, v[i + 2] * qs, v[i + 3] * qs);
        w.y = pack4_e4m3(v[i + 4] * qs, v[i + 5] * qs, v[i + 6] * qs, v[i + 7] * qs);
        *reinterpret_cast<uint2*>(dst + i) = w;
      }
    } else {
#pragma unroll
      for (int i = 0; i < EPL; i += 4)
        *reinterpret_cast<float4*>(dst + 4 * i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
    }
  }
  {  // h rows of symbols -1 and 14 (rows t in [T, 14) were written as zeros above)
    constexpr int CH = C * (int)sizeof(Op) / 16;  // 16-byte chunks per position
    for (int i = threadIdx.x; i < 2 * HW * CH; i += NT) {
      const int rr = i / (HW * CH), rem = i - rr * HW * CH;
      const int j = rem / CH, ch = rem - j * CH;
      *reinterpret_cast<i32x4*>(lds + ((rr ? TROWS - 1 : 0) * HW + j) * PITCH + ch * 16) = i32x4{0, 0, 0, 0};
    }
  }
  __syncthreads();

  // 4. conv 2 on RE q = t * TWO + j of the output region (symbol t, subcarrier f0 + j).
  //    The block output's other inputs (the residual x and, on the main branch, the
  //    support outputs) of the first PRE M-tiles are loaded into registers while the
  //    MFMAs run; the rest are issued right after (all of them on a plain branch, then
  //    PD M-tiles ahead on the main branch).
  using RawT = RawOf<Act, EPL>;
  constexpr int NR = EPL * (int)sizeof(Act) / (int)sizeof(RawT);
  constexpr int NTEN = 1 + NSUP;
  constexpr int PDM = (OCC >= 3 && NSUP >= 2) ? 1 : 2;  // at three per CU the registers hold one M-tile
  constexpr int PD = (MAIN || OCC >= 3) ? (MT2 < PDM ? MT2 : PDM) : (MT2 < 4 ? MT2 : 4);
  RawT raw[PD][NTEN][NR];
  auto re_of = [&](int mt, bool& ok) -> int64_t {
    const int q = (wave + NW * mt) * 16 + col;
    const int t = q / TWO, j = q - t * TWO;
    const int f = td.f0 + j;
    ok = wave + NW * mt < M2 && q < Q2 && t < T && f < td.F;
    return td.re_base + (int64_t)t * td.F + f;
  };
  auto issue = [&](int mt) {
    bool ok;
    int64_t re = re_of(mt, ok);
    if (!ok) re = td.re_base;  // any RE of the slot: loaded, never used
    const RawT* p = reinterpret_cast<const RawT*>(reinterpret_cast<const Act*>(args.x[k]) + re * C + c0);
#pragma unroll
    for (int r = 0; r < NR; ++r) raw[mt % PD][0][r] = p[r];
#pragma unroll
    for (int sidx = 1; sidx <= NSUP; ++sidx) {
      const RawT* ps_ = reinterpret_cast<const RawT*>(reinterpret_cast<const Act*>(args.sup[sidx]) + re * C + c0);
#pragma unroll
      for (int r = 0; r < NR; ++r) raw[mt % PD][sidx][r] = ps_[r];
    }
  };
  constexpr int PRE = OCC >= 3 ? 0 : MAIN ? 1 : (PD < 2 ? PD : 2);  // as the GEMM's registers allow
#pragma unroll
  for (int d = 0; d < PRE; ++d) issue(d);
  AccV acc2[MT2][NOT];
  {
    int base[MT2];
#pragma unroll
    for (int mt = 0; mt < MT2; ++mt) {
      int q = (wave + NW * mt) * 16 + col;
      if (q >= Q2) q = Q2 - 1;
      const int t = q / TWO, j = q - t * TWO;
      base[mt] = (t * HW + j) * PITCH;  // tap (-1, -1): h row t (symbol t - 1), column j
    }
    G2::run(acc2, lds, reinterpret_cast<const i32x4*>(args.w2[k]), base, lane);
  }
#pragma unroll
  for (int d = PRE; d < PD; ++d) issue(d);
#pragma unroll
  for (int i = 0; i < EPL; ++i) {
    pb[i] = par[P_B2 * C + c0 + i];
    pq[i] = par[P_Q2 * C + c0 + i];
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
#pragma unroll
  for (int mt = 0; mt < MT2; ++mt) {
    bool ok;
    const int64_t re = re_of(mt, ok);
    if (ok) {
      Acc v[EPL];
#pragma unroll
      for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          Acc a = acc2[mt][ot][i];
          if constexpr (A::QUANT) a = a * (Acc)pq[4 * ot + i];
          v[4 * ot + i] = a + (Acc)pb[4 * ot + i];
        }
      finish_block<A, C, EPL, NSUP>(
          v, re, c0, g, MAIN, [&](Acc* x) { unpack_raw<Act, RawT, EPL>(raw[mt % PD][0], x); },
          [&](int kk, Acc* sv) { unpack_raw<Act, RawT, EPL>(raw[mt % PD][kk], sv); }, MAIN ? args.out[0] : args.out[k],
          (MAIN || k == 0) ? args.save_o0 : nullptr, head, NSUP + 1, par + P_GAM * C, par + P_BET * C, args.eps, whl, whl + args.m * C, args.llr,
          args.m, args.fusion_sum != 0, (MAIN && args.feedback) ? const_cast<void* const*>(args.sup) : nullptr,
          args.norm_affine != 0);
    }
    if (mt + PD < MT2) issue(mt + PD);
  }
}

// One fused block per work-group: branch blockIdx.y + k_off.
template <class A, int C, int TWO, bool MAIN, bool HEAD, int NSUP>
__global__ void __launch_bounds__(CONV_NW * 64, (block_occ<A, C, TWO>())) block_kernel(BlockArgs args) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[block_lds_bytes<A, C, TWO>()];
  block_body<A, C, TWO, MAIN, HEAD, NSUP>(args, blockIdx.y + args.k_off, lds, xcd_remap(blockIdx.x, gridDim.x));
}

// The main branch of block l (branch 0, fusion epilogue over the supports' stored outputs of
// block l) together with the support branches of block l + 1 (branches >= 1, which read only
// the supports' outputs of block l): independent work in one launch. The per-branch argument
// arrays carry block l for branch 0 and block l + 1 for the others. The grid is (tiles, K).
// A launch of at least PAIR_TILE_MAJOR work-groups (eight rounds of two per CU on 256 CUs) takes
// them in dispatch order and maps consecutive ones to the K branches of one tile, contiguous runs
// of tiles per XCD: every CU holds a mix of the heavier main-branch epilogues and the support
// branches, and a tile's branches, which read the same support outputs of block l, share an XCD's
// L2 (on the 64-slot batch: 3.44 instead of 4.15 GB from HBM, 1.5 % faster). A smaller launch
// keeps a branch per grid row: at one slot the tile-major order measured 4.5 % slower.
constexpr int PAIR_TILE_MAJOR = 4096;
template <class A, int C, int TWO, int NSUP>
__global__ void __launch_bounds__(CONV_NW * 64, (block_occ<A, C, TWO>())) block_pair_kernel(BlockArgs args) {
  __shared__ __attribute__((aligned(16))) uint8_t lds[block_lds_bytes<A, C, TWO>()];
  const int K = gridDim.y, n = gridDim.x * K;
  int tile, k;
  if (n >= PAIR_TILE_MAJOR) {
    const int r = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, n);
    tile = r / K;
    k = r - tile * K;
  } else {
    tile = xcd_remap(blockIdx.x, gridDim.x);
    k = blockIdx.y;
  }
  if (k == 0)
    block_body<A, C, TWO, true, false, NSUP>(args, 0, lds, tile);
  else
    block_body<A, C, TWO, false, false, 0>(args, k, lds, tile);
}

template <class A, int C, int TWO, bool HEAD>
static hipError_t launch_block_h(int kind, BlockArgs& a, dim3 grid, hipStream_t s) {
  const dim3 blk(CONV_NW * 64);
  if (kind == BLOCK_PLAIN) {
    hipLaunchKernelGGL((block_kernel<A, C, TWO, false, HEAD, 0>), grid, blk, 0, s, a);
  } else if (kind == BLOCK_MAIN) {
    switch (a.K) {
      case 1: hipLaunchKernelGGL((block_kernel<A, C, TWO, true, HEAD, 0>), grid, blk, 0, s, a); break;
      case 2: hipLaunchKernelGGL((block_kernel<A, C, TWO, true, HEAD, 1>), grid, blk, 0, s, a); break;
      case 3: hipLaunchKernelGGL((block_kernel<A, C, TWO, true, HEAD, 2>), grid, blk, 0, s, a); break;
      case 4: hipLaunchKernelGGL((block_kernel<A, C, TWO, true, HEAD, 3>), grid, blk, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  } else {  // BLOCK_PAIR: no head (the last block's main branch runs alone)
    if constexpr (HEAD) return hipErrorInvalidValue;
    switch (a.K) {
      case 2: hipLaunchKernelGGL((block_pair_kernel<A, C, TWO, 1>), grid, blk, 0, s, a); break;
      case 3: hipLaunchKernelGGL((block_pair_kernel<A, C, TWO, 2>), grid, blk, 0, s, a); break;
      case 4: hipLaunchKernelGGL((block_pair_kernel<A, C, TWO, 3>), grid, blk, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <class A, int C, int TWO>
static hipError_t launch_block_w(int kind, BlockArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  a.tw = TWO;
  if (a.llr && (a.m < 1 || a.m > 8)) return hipErrorInvalidValue;
  const dim3 grid(n_tiles, grid_y);
  return a.llr ? launch_block_h<A, C, TWO, true>(kind, a, grid, s) : launch_block_h<A, C, TWO, false>(kind, a, grid, s);
}

template <class A, int C>
static hipError_t launch_block_c(int kind, int wclass, BlockArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  constexpr int TW = block_tw<A, C, TW_WIDE>(), TN = block_tw<A, C, TW_NARROW>(), T3 = block_tw<A, C, TW_NARROW3>();
  if constexpr (TW == 0) {
    return hipErrorInvalidValue;
  } else {
    if (wclass == TW_NARROW3) {
      if constexpr (T3 != 0) return launch_block_w<A, C, T3>(kind, a, n_tiles, grid_y, s);
      return hipErrorInvalidValue;
    }
    if constexpr (TN != TW) {
      if (wclass == TW_NARROW) return launch_block_w<A, C, TN>(kind, a, n_tiles, grid_y, s);
    }
    return launch_block_w<A, C, TW>(kind, a, n_tiles, grid_y, s);
  }
}

template <class A>
hipError_t launch_block_dtype(int kind, int wclass, int C, BlockArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  switch (C) {
    case 16: return launch_block_c<A, 16>(kind, wclass, a, n_tiles, grid_y, s);
    case 32: return launch_block_c<A, 32>(kind, wclass, a, n_tiles, grid_y, s);
    case 64: return launch_block_c<A, 64>(kind, wclass, a, n_tiles, grid_y, s);
  }
  return hipErrorInvalidValue;
}

template <class A>
int block_tile_width_dtype(int C, int wclass) {
  auto pick = [wclass](int w, int n, int n3) { return wclass == TW_NARROW3 ? n3 : wclass == TW_NARROW ? n : w; };
  switch (C) {
    case 16: return pick(block_tw<A, 16>(), block_tw<A, 16, TW_NARROW>(), block_tw<A, 16, TW_NARROW3>());
    case 32: return pick(block_tw<A, 32>(), block_tw<A, 32, TW_NARROW>(), block_tw<A, 32, TW_NARROW3>());
    case 64: return pick(block_tw<A, 64>(), block_tw<A, 64, TW_NARROW>(), block_tw<A, 64, TW_NARROW3>());
  }
  return 0;
}

}  // namespace conet
