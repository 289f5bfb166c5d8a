// Input gradient of one residual block in one launch (BF16, gfx950): the adjoint of the fused
// forward block in conet_block_impl.h.
//
// The forward block is O = x + W2 * h + b2 with h = ReLU(s1 (W1 * pre(x) + b1) + o1) and
// pre(x) = ReLU(s0 x + o0) (ReLU(x) on the main branch after a fusion). Reverse mode gives
//   dz1 = [h > 0] (W2^T * dO),   dc1 = s1 dz1,
//   dz0 = [s0 x + o0 > 0] (W1^T * dc1),   dx = dO + s0 dz0,
// where W^T * is the 3x3 conv with the filter transposed in channels and flipped in space
// (its own fragment pack). Run as two convs, dc1 makes a round trip through HBM and every
// work-group stages a halo tile per conv; here one work-group owns one tile (a slot, its
// T <= 14 symbols, TWO subcarriers) and:
//   1. stages dO for subcarriers f0-2 .. f0+TWO+1 (two-RE halo) into LDS,
//   2. runs W2^T on the 14 x (TWO+2) region that the second transposed conv needs,
//   3. after a barrier, overwrites the dO tile with dc1 (zero outside the slot, rounded to
//      the activation type exactly as a stored dc1 would be), stores the tile's own dc1 (the
//      filter gradient of conv 1 reads it) and sums the s1 / o1 gradients over its own REs,
//   4. runs W1^T on the 14 x TWO output region and finishes dx and the s0 / o0 gradient sums.
// The arithmetic per RE is that of the two-conv path, so dc1 and dx are bit-identical to it;
// only the grouping of the per-channel partial sums differs (other tiles).
#include "conet_block_impl.h"
#include "conet_bwd_block.h"

namespace conet {

template <class A, int C, int TWO>
__global__ void __launch_bounds__(CONV_NW * 64, 2) bwd_block_kernel(BwdBlockArgs args) {
  using AccV = typename A::AccV;
  using Act = typename A::Act;
  using Op = typename A::Op;
  static_assert(sizeof(Op) == 2 && std::is_same<Act, Op>::value, "BF16 operands and activations");
  constexpr int NW = CONV_NW, NT = NW * 64;
  constexpr int XW = TWO + 4, HW = TWO + 2;  // LDS positions per row: dO tile, dc1 tile
  constexpr int PITCH = lds_pitch<A, C>();
  constexpr int Q1 = TMAX * HW, Q2 = TMAX * TWO;  // REs of the two conv regions
  constexpr int M1 = (Q1 + 15) / 16, M2 = (Q2 + 15) / 16;
  constexpr int MT1 = (M1 + NW - 1) / NW, MT2 = (M2 + NW - 1) / NW;
  constexpr int NOT = C / 16, EPL = 4 * NOT;
  constexpr int TILE = TROWS * XW * PITCH;
  enum { P_S1, P_O1, P_S0, P_O0, NP };
  using G1 = GemmCore<A, C, C, XW, PITCH, MT1, 200>;
  using G2 = GemmCore<A, C, C, HW, PITCH, MT2, 200>;
  static_assert(2 * (TILE + NP * C * 4) <= 160 * 1024, "LDS must leave room for two work-groups per CU");
  static_assert((EPL * (int)sizeof(Act)) % 16 == 0, "a lane's channels fill whole 16-byte words");
  __shared__ __attribute__((aligned(16))) uint8_t lds[TILE + NP * C * 4];
  float* par = reinterpret_cast<float*>(lds + TILE);

  const int k = blockIdx.y;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const TileDesc td = tile_of(args, bid);
  const int T = args.T;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, col = lane & 15;
  const int c0 = g * EPL;  // first channel owned by this lane
  const bool mrb = args.s0[k] == nullptr;

  // 0. per-channel parameters: loads issued now, written to LDS after the tile's loads
  constexpr int NPV = (NP * C + NT - 1) / NT;
  float pv[NPV];
#pragma unroll
  for (int u = 0; u < NPV; ++u) {
    const int i = threadIdx.x + u * NT;
    const int pi = i / C, c = i - pi * C;
    float val = 0.f;
    switch (pi) {
      case P_S1: val = args.s1[k][c]; break;
      case P_O1: val = args.o1[k][c]; break;
      case P_S0: val = mrb ? 1.f : args.s0[k][c]; break;
      case P_O0: val = mrb ? 0.f : args.o0[k][c]; break;
      default: break;
    }
    pv[u] = val;
  }

  // 1. dO with a two-RE halo; LDS row r = symbol r - 1, column c = subcarrier f0 + c - 2
  stage_tile<A, Act, C, XW, 2, PITCH, NT>(lds, reinterpret_cast<const Act*>(args.dO[k]), td, T, 0, nullptr, nullptr,
                                          1.f);
#pragma unroll
  for (int u = 0; u < NPV; ++u)
    if (threadIdx.x + u * NT < NP * C) par[threadIdx.x + u * NT] = pv[u];
  __syncthreads();

  // 2. W2^T on RE q = t * HW + j of the region (symbol t, subcarrier f0 - 1 + j). The mask
  //    operand h of the first M-tile is loaded before the MFMAs, those of the others right
  //    after them, all into registers at once, so their latencies overlap.
  constexpr int NR = EPL * (int)sizeof(Act) / 16;
  i32x4 hr[MT1][NR];
  auto h_at = [&](int mt, int& t, int& j, bool& valid) -> int64_t {
    const int q = (wave + NW * mt) * 16 + col;
    t = q / HW;
    j = q - t * HW;
    const int f = td.f0 - 1 + j;
    valid = wave + NW * mt < M1 && q < Q1 && t < T && f >= 0 && f < td.F;
    return td.re_base + (int64_t)t * td.F + f;
  };
  auto load_h = [&](int mt) {
    int t, j;
    bool valid;
    int64_t re = h_at(mt, t, j, valid);
    if (!valid) re = td.re_base;  // any RE of the slot: loaded, never used
    const i32x4* p = reinterpret_cast<const i32x4*>(reinterpret_cast<const Act*>(args.h[k]) + re * C + c0);
#pragma unroll
    for (int r = 0; r < NR; ++r) hr[mt][r] = p[r];
  };
  AccV acc1[MT1][NOT];
  {
    int base[MT1];
#pragma unroll
    for (int mt = 0; mt < MT1; ++mt) {
      int q = (wave + NW * mt) * 16 + col;
      if (q >= Q1) q = Q1 - 1;  // surplus lanes recompute a real RE (never written)
      const int t = q / HW, j = q - t * HW;
      base[mt] = (t * XW + j) * PITCH;  // tap (-1, -1): dO row t (symbol t - 1), column j
    }
    load_h(0);
    G1::run(acc1, lds, reinterpret_cast<const i32x4*>(args.wt2[k]), base, lane);
  }
#pragma unroll
  for (int mt = 1; mt < MT1; ++mt) load_h(mt);

  // 3. dc1 = s1 [h > 0] dh, formed in place of the accumulators one group of four channels at
  //    a time (the group's affine and sums in registers), with the s1 / o1 gradient sums over
  //    this tile's own REs; then written into LDS row t + 1 (symbol t), column j, zero for REs
  //    outside the slot (the second transposed conv's zero padding), and stored for the
  //    tile's own REs.
  auto region_re = [&](int mt, int& t, int& j, bool& live, bool& valid) -> int64_t {
    const int q = (wave + NW * mt) * 16 + col;
    live = wave + NW * mt < M1 && q < Q1;
    return h_at(mt, t, j, valid);
  };
  float* row1 = args.part[k] + ((size_t)blockIdx.x * NW + wave) * 3 * C;
#pragma unroll
  for (int ot = 0; ot < NOT; ++ot) {
    float s1v[4], o1v[4], sa[4], sb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s1v[i] = par[P_S1 * C + c0 + 4 * ot + i];
      o1v[i] = par[P_O1 * C + c0 + 4 * ot + i];
      sa[i] = 0.f;
      sb[i] = 0.f;
    }
#pragma unroll
    for (int mt = 0; mt < MT1; ++mt) {
      int t, j;
      bool live, valid;
      region_re(mt, t, j, live, valid);
      const bool own = live && valid && j >= 1 && j <= TWO;  // this tile's own REs carry the sums
      const Act* hv = reinterpret_cast<const Act*>(hr[mt]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float h = (float)hv[4 * ot + i];
        const float dz = h > 0.f ? (float)acc1[mt][ot][i] : 0.f;
        acc1[mt][ot][i] = valid ? dz * s1v[i] : 0.f;
        if (own) {
          sa[i] += dz * (h - o1v[i]);  // divided by s1 once, after the sums
          sb[i] += dz;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // over the 16 lanes that hold the same channels
      float a = sa[i], b = sb[i];
      a += __shfl_xor(a, 1);
      a += __shfl_xor(a, 2);
      a += __shfl_xor(a, 4);
      a += __shfl_xor(a, 8);
      b += __shfl_xor(b, 1);
      b += __shfl_xor(b, 2);
      b += __shfl_xor(b, 4);
      b += __shfl_xor(b, 8);
      if (col == 0) {
        row1[c0 + 4 * ot + i] = a / s1v[i];
        row1[C + c0 + 4 * ot + i] = b;
      }
    }
  }
  __syncthreads();  // every wave has read its last dO operand: dc1 may overwrite the tile
#pragma unroll
  for (int mt = 0; mt < MT1; ++mt) {
    int t, j;
    bool live, valid;
    const int64_t re = region_re(mt, t, j, live, valid);
    if (!live) continue;
    float v[EPL];
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int i = 0; i < 4; ++i) v[4 * ot + i] = acc1[mt][ot][i];
    if (valid && j >= 1 && j <= TWO) store_vals(reinterpret_cast<Act*>(args.dc1[k]) + re * C + c0, v, EPL, 1.f);
    uint8_t* dst = lds + ((t + 1) * HW + j) * PITCH + c0 * (int)sizeof(Op);
#pragma unroll
    for (int i = 0; i < EPL; i += 8) {
      __bf16 bb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) bb[u] = f2bf(v[i + u]);
      *reinterpret_cast<i32x4*>(dst + 2 * i) = *reinterpret_cast<const i32x4*>(bb);
    }
  }
  {  // dc1 rows of symbols -1 and 14 (rows t in [T, 14) were written as zeros above)
    constexpr int CH = C * (int)sizeof(Op) / 16;  // 16-byte chunks per position
    for (int i = threadIdx.x; i < 2 * HW * CH; i += NT) {
      const int rr = i / (HW * CH), rem = i - rr * HW * CH;
      const int j = rem / CH, ch = rem - j * CH;
      *reinterpret_cast<i32x4*>(lds + ((rr ? TROWS - 1 : 0) * HW + j) * PITCH + ch * 16) = i32x4{0, 0, 0, 0};
    }
  }
  __syncthreads();

  // 4. W1^T on RE q = t * TWO + j of the output region (symbol t, subcarrier f0 + j). The
  //    epilogue's operands x and dO are loaded into registers PD M-tiles ahead (the first
  //    while the MFMAs run).
  constexpr int PD = MT2 < 2 ? MT2 : 2;
  i32x4 raw[PD][2][NR];
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
    if (!ok) re = td.re_base;
    const i32x4* px = reinterpret_cast<const i32x4*>(reinterpret_cast<const Act*>(args.x[k]) + re * C + c0);
    const i32x4* pd = reinterpret_cast<const i32x4*>(reinterpret_cast<const Act*>(args.dO[k]) + re * C + c0);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      raw[mt % PD][0][r] = px[r];
      raw[mt % PD][1][r] = pd[r];
    }
  };
  issue(0);
  AccV acc2[MT2][NOT];
  {
    int base[MT2];
#pragma unroll
    for (int mt = 0; mt < MT2; ++mt) {
      int q = (wave + NW * mt) * 16 + col;
      if (q >= Q2) q = Q2 - 1;
      const int t = q / TWO, j = q - t * TWO;
      base[mt] = (t * HW + j) * PITCH;  // tap (-1, -1): dc1 row t (symbol t - 1), column j
    }
    G2::run(acc2, lds, reinterpret_cast<const i32x4*>(args.wt1[k]), base, lane);
  }
#pragma unroll
  for (int d = 1; d < PD; ++d) issue(d);
  float ps[EPL], po[EPL], sa[EPL], sb[EPL];
#pragma unroll
  for (int i = 0; i < EPL; ++i) {
    ps[i] = par[P_S0 * C + c0 + i];
    po[i] = par[P_O0 * C + c0 + i];
    sa[i] = 0.f;
    sb[i] = 0.f;
  }
  const bool mask_out = args.mask_out != 0;
#pragma unroll
  for (int mt = 0; mt < MT2; ++mt) {
    bool ok;
    const int64_t re = re_of(mt, ok);
    if (ok) {
      const Act* xv = reinterpret_cast<const Act*>(raw[mt % PD][0]);
      const Act* dv = reinterpret_cast<const Act*>(raw[mt % PD][1]);
      float v[EPL];
#pragma unroll
      for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int e = 4 * ot + i;
          const float x = (float)xv[e], dO = (float)dv[e];
          const float z0 = ps[e] * x + po[e];
          const float dz = z0 > 0.f ? (float)acc2[mt][ot][i] : 0.f;
          float dx = dO + ps[e] * dz;
          if (mask_out && !(x > 0.f)) dx = 0.f;
          sa[e] += mrb ? 0.f : dz * x;
          sb[e] += mrb ? 0.f : dz;
          v[e] = dx;
        }
      store_vals(reinterpret_cast<Act*>(args.dx[k]) + re * C + c0, v, EPL, 1.f);
    }
    if (mt + PD < MT2) issue(mt + PD);
  }
#pragma unroll
  for (int i = 0; i < EPL; ++i) {  // over the 16 lanes that hold the same channels
    float a = sa[i], b = sb[i];
    a += __shfl_xor(a, 1);
    a += __shfl_xor(a, 2);
    a += __shfl_xor(a, 4);
    a += __shfl_xor(a, 8);
    b += __shfl_xor(b, 1);
    b += __shfl_xor(b, 2);
    b += __shfl_xor(b, 4);
    b += __shfl_xor(b, 8);
    sa[i] = a;
    sb[i] = b;
  }
  if (col == 0) {
    float* row0 = args.part[k] + ((size_t)args.rows + (size_t)blockIdx.x * NW + wave) * 3 * C;
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      row0[c0 + i] = sa[i];
      row0[C + c0 + i] = sb[i];
    }
  }
}

template <class A, int C>
static hipError_t launch_bwd_c(BwdBlockArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  constexpr int TWO = block_tw<A, C>();
  a.tw = TWO;
  a.tiles = nullptr;
  hipLaunchKernelGGL((bwd_block_kernel<A, C, TWO>), dim3(n_tiles, grid_y), dim3(CONV_NW * 64), 0, s, a);
  return hipGetLastError();
}

int bwd_block_tile_width(int dtype, int C) {
  if (dtype != DT_BF16) return 0;
  if (C == 32) return block_tw<ArithBF16, 32>();
  if (C == 64) return block_tw<ArithBF16, 64>();
  return 0;
}

hipError_t launch_bwd_block(int dtype, int C, BwdBlockArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  if (dtype != DT_BF16 || n_tiles <= 0 || grid_y <= 0 || grid_y > KMAX_ARGS) return hipErrorInvalidValue;
  if (C == 32) return launch_bwd_c<ArithBF16, 32>(a, n_tiles, grid_y, s);
  if (C == 64) return launch_bwd_c<ArithBF16, 64>(a, n_tiles, grid_y, s);
  return hipErrorInvalidValue;
}

}  // namespace conet
