// 3x3 implicit-GEMM convolution kernels of the CoNet-Rx forward pass (gfx950).
//
// One work-group owns one tile: a slot, all of its T <= 14 OFDM symbols and TW
// consecutive subcarriers, for one branch. The tile's input (with a one-RE zero halo
// on every side, padding taken inside the slot) is staged once into LDS in the MFMA
// operand type; the pre-activation prologue (affine + ReLU, or ReLU) and FP8
// quantisation are applied while staging. Each wave then runs the GEMM
//     D^T[o, re] = sum_k W[o, k] * X^T[k, re],   k = (tap, channel)
// on 16x16 MFMA tiles: the A operand is the filter, pre-packed on the host in the
// exact per-lane fragment order (one coalesced 16-byte load per lane, prefetched one
// K step ahead), and the B operand is read from LDS as 16-byte chunks of consecutive
// channels at the tap-shifted position. The epilogue works on FP32 accumulators:
// bias, per-channel affine, ReLU, residual add, the K-way product fusion with the
// per-RE channel LayerNorm, and the 1x1 LLR head.
//
// Output channel ownership: within o-tile `ot`, MFMA row r = 4g + i (g = lane/16)
// holds channel g*4*NOT + 4*ot + i, so every lane owns 4*NOT consecutive channels of
// one RE and stores them with wide vector writes. The host packs filters with the
// same permutation.
//
// Register budget: every kernel is built for two work-groups per CU (<= 256 VGPR +
// AGPR per lane, LDS tile <= 80 KB), so one work-group's staging overlaps the other's
// MFMA loop.
#pragma once
#include "conet_common.h"
#include "conet_kernels.h"

namespace conet {

// ---------------------------------------------------------------- vector IO helpers
template <class T>
__device__ __forceinline__ void load_vals(const T* p, float* v, int n) {
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
template <class Args>
__device__ __forceinline__ TileDesc tile_of(const Args& a, int bid) {
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

// ---------------------------------------------------------------- shapes
template <class A, int CIN>
constexpr int lds_pitch() {
  int p = CIN * (int)sizeof(typename A::Op);
  return ((p / 16) % 2 == 0) ? p + 16 : p;  // odd multiple of 16 B: conflict-free 16-B reads
}

// 32 subcarriers per tile unless the halo tile would not leave room for two
// work-groups per CU, or the channel count would exceed the per-lane register budget.
template <class A, int CIN, int COUT>
constexpr int tile_w() {
  return (COUT > 64 || TROWS * 34 * lds_pitch<A, CIN>() > 80 * 1024) ? 16 : 32;
}

// ---------------------------------------------------------------- staging
// Stage the TROWS x XW halo tile of `in` (CIN channels of InT per RE) into LDS as Op
// with PITCH bytes per position: LDS row r holds OFDM symbol r - 1, column c holds
// subcarrier f0 + c - COFF. Thread `tid` always handles the same channel chunk (its
// prologue parameters stay in registers); loads are issued in batches of NB positions
// before any is consumed, so their latencies overlap.
template <class A, class InT, int CIN, int XW, int COFF, int PITCH, int NT>
__device__ __forceinline__ void stage_tile(uint8_t* lds, const InT* __restrict__ in, const TileDesc& td, int T,
                                           int prologue, const float* __restrict__ ps, const float* __restrict__ po,
                                           float qscale) {
  using Op = typename A::Op;
  constexpr int EPC = 16 / sizeof(InT) < 4 ? 4 : 16 / (int)sizeof(InT);  // elements per 16-B global chunk
  constexpr int CPP = CIN / EPC;                                          // chunks per position
  constexpr int NPOS = TROWS * XW;
  constexpr int PPR = NT / CPP;                                           // positions per round
  constexpr int NIT = (NPOS + PPR - 1) / PPR;
  constexpr int NB = NIT <= 24 ? NIT : 8;  // all of a thread's loads in flight at once when they fit
  static_assert(CIN % EPC == 0 && sizeof(InT) <= 4, "channel count must fill whole 16-byte chunks");
  const int tid = threadIdx.x;
  if (tid >= PPR * CPP) return;
  const int cc = tid % CPP, p0 = tid / CPP, ch = cc * EPC;
  constexpr bool COPY = std::is_same<InT, Op>::value;
  float sv[EPC], ov[EPC];
  if (prologue == 1) {
#pragma unroll
    for (int i = 0; i < EPC; ++i) { sv[i] = ps[ch + i]; ov[i] = po[ch + i]; }
  }
#pragma unroll 1
  for (int b0 = 0; b0 < NIT; b0 += NB) {
    i32x4 raw[NB];
    bool ok[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int pos = p0 + (b0 + j) * PPR;
      const int r = pos / XW, c = pos - r * XW;
      const int t = r - 1, f = td.f0 + c - COFF;
      ok[j] = (b0 + j < NIT) && pos < NPOS && t >= 0 && t < T && f >= 0 && f < td.F;
      raw[j] = i32x4{0, 0, 0, 0};
      if (ok[j]) raw[j] = *reinterpret_cast<const i32x4*>(in + (td.re_base + (int64_t)t * td.F + f) * CIN + ch);
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int pos = p0 + (b0 + j) * PPR;
      if (b0 + j >= NIT || pos >= NPOS) continue;
      uint8_t* dst = lds + pos * PITCH + ch * (int)sizeof(Op);
      if constexpr (COPY) {
        if (prologue == 0) {  // stored in the operand type already (zero where out of the slot)
          *reinterpret_cast<i32x4*>(dst) = raw[j];
          continue;
        }
      }
      float v[EPC];
      const InT* rv = reinterpret_cast<const InT*>(&raw[j]);
#pragma unroll
      for (int i = 0; i < EPC; ++i) v[i] = (float)rv[i];
      if (prologue == 1) {
#pragma unroll
        for (int i = 0; i < EPC; ++i) v[i] = fmaxf(sv[i] * v[i] + ov[i], 0.f);
      } else if (prologue == 2) {
#pragma unroll
        for (int i = 0; i < EPC; ++i) v[i] = fmaxf(v[i], 0.f);
      }
      if (!ok[j]) {
#pragma unroll
        for (int i = 0; i < EPC; ++i) v[i] = 0.f;  // zero padding applies after the prologue
      }
      if constexpr (sizeof(Op) == 1) {
#pragma unroll
        for (int i = 0; i < EPC; i += 4)
          *reinterpret_cast<uint32_t*>(dst + i) =
              pack4_e4m3(v[i] * qscale, v[i + 1] * qscale, v[i + 2] * qscale, v[i + 3] * qscale);
      } else if constexpr (sizeof(Op) == 2) {
#pragma unroll
        for (int i = 0; i < EPC; i += 4) {
          __bf16 bb[4] = {f2bf(v[i]), f2bf(v[i + 1]), f2bf(v[i + 2]), f2bf(v[i + 3])};
          *reinterpret_cast<uint2*>(dst + 2 * i) = *reinterpret_cast<const uint2*>(bb);
        }
      } else {
#pragma unroll
        for (int i = 0; i < EPC; i += 4)
          *reinterpret_cast<float4*>(dst + 4 * i) = make_float4(v[i], v[i + 1], v[i + 2], v[i + 3]);
      }
    }
  }
}

// Stage the input layer's halo tile straight from the received grid y (FP32 [RE][n_rx][2]):
// the features of every position -- Re y, Im y and the LS channel estimate interpolated to
// its symbol, per antenna, zeros for antennas n_rx .. CIN/4 - 1 -- are formed on the fly with
// the featuriser's own steps (bit-identical to conet_featurise), then rounded to Op. One
// thread per (antenna group, position); the pilot-row samples a column needs are re-read
// from cache by the 16 rows that use them. Needs T >= 12 (both pilot symbols).
template <class A, int CIN, int XW, int COFF, int PITCH, int NT>
__device__ __forceinline__ void stage_grid_tile(uint8_t* lds, const float2* __restrict__ y, const TileDesc& td, int T,
                                                int n_rx, float qscale) {
  using Op = typename A::Op;
  constexpr int CPP = CIN / 4;  // antenna groups per position
  constexpr int NPOS = TROWS * XW;
  constexpr int PPR = NT / CPP;
  const int tid = threadIdx.x;
  if (tid >= PPR * CPP) return;
  const int n = tid % CPP, p0 = tid / CPP;
  const float2* __restrict__ slot = y + td.re_base * n_rx + n;  // antenna n's sample of (t = 0, f = 0)
  for (int pos = p0; pos < NPOS; pos += PPR) {
    const int r = pos / XW, c = pos - r * XW;
    const int t = r - 1, f = td.f0 + c - COFF;
    float v[4] = {0.f, 0.f, 0.f, 0.f};
    if (n < n_rx && t >= 0 && t < T && f >= 0 && f < td.F) {
      const float2 yv = slot[((int64_t)t * td.F + f) * n_rx];
      const float2 h0 = pilot_row_estimate(slot + (int64_t)PILOT_T0 * td.F * n_rx, n_rx, f, td.F);
      const float2 h1 = pilot_row_estimate(slot + (int64_t)PILOT_T1 * td.F * n_rx, n_rx, f, td.F);
      const float2 h = interp_symbol(h0, h1, t);
      v[0] = yv.x; v[1] = yv.y; v[2] = h.x; v[3] = h.y;
    }
    uint8_t* dst = lds + pos * PITCH + 4 * n * (int)sizeof(Op);
    if constexpr (sizeof(Op) == 1) {
      *reinterpret_cast<uint32_t*>(dst) = pack4_e4m3(v[0] * qscale, v[1] * qscale, v[2] * qscale, v[3] * qscale);
    } else if constexpr (sizeof(Op) == 2) {
      __bf16 bb[4] = {f2bf(v[0]), f2bf(v[1]), f2bf(v[2]), f2bf(v[3])};
      *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(bb);
    } else {
      *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
    }
  }
}

// ---------------------------------------------------------------- GEMM core
// acc[mt][ot] += W (o-tile ot) x X^T (M-tile mt) over all K steps, for MT M-tiles of
// 16 REs each. The caller gives, per M-tile, the LDS byte offset of this lane's RE for
// tap (-1, -1); the staged input has ROWP positions per row and PITCH bytes per
// position, so tap (dt, dc) adds ((dt + 1) ROWP + dc + 1) positions.
template <class A, int CIN, int COUT, int ROWP, int PITCH, int MT, int VBUDGET = 200>
struct GemmCore {
  static constexpr int NOT = COUT / 16;
  static constexpr int CPT = CIN / A::VEC;                       // chunks per tap
  static constexpr int NCH = 9 * CPT;                            // real chunks
  static constexpr int CPS = 4 * A::CPL;                         // chunks per K step
  static constexpr int NS = (NCH + CPS - 1) / CPS;               // K steps
  static_assert(COUT % 16 == 0, "output channels must be a multiple of 16");
  static_assert(CIN % A::VEC == 0, "");

  using AccV = typename A::AccV;

  __device__ __forceinline__ static void load_a(i32x4 (&a)[NOT][A::CPL], const i32x4* __restrict__ wp, int s,
                                                int lane) {
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int c = 0; c < A::CPL; ++c) a[ot][c] = wp[((s * NOT + ot) * A::CPL + c) * 64 + lane];
  }

  // LDS byte offset of this lane's B fragment (chunk c of K step s) relative to its
  // M-tile base: the step's tap shift plus 16 bytes of consecutive channels
  __device__ __forceinline__ static constexpr int b_off(int s, int c, int g) {
    int ch = (s * 4 + g) * A::CPL + c;
    if (ch >= NCH) ch = 4 * CPT;  // padding chunk: any in-tile address (its weights are 0)
    const int tap = ch / CPT, c0 = (ch - tap * CPT) * A::VEC;
    return ((tap / 3) * ROWP + (tap % 3)) * PITCH + c0 * (int)sizeof(typename A::Op);
  }

  // Filter fragments are prefetched ADEPTH K steps ahead (a ring of ADEPTH + 1 buffers)
  // when the registers allow it (VBUDGET VGPRs for accumulators and operands), else one
  // step ahead.
  static constexpr int ADEPTH = (MT * NOT * 4 + 3 * NOT * A::CPL * 4 + MT * A::CPL * 4 <= VBUDGET) ? 2 : 1;
  // B fragments are prefetched unless two chunks per MFMA (FP8) leave no registers for it;
  // then each step issues its own B reads first. BF16 prefetches through a ring of three
  // buffers, FP32 one step ahead in one buffer per M-tile (the ring measured 1.6 % faster
  // on the BF16 forward and 60 % slower on the FP32 one at 96 channels).
  enum { B_PLAIN, B_ROLL, B_RING };
  static constexpr int BMODE = A::CPL != 1 ? B_PLAIN : sizeof(typename A::Op) == 2 ? B_RING : B_ROLL;

  __device__ __forceinline__ static void load_b(i32x4 (&b)[A::CPL], const uint8_t* lds, int base, int s, int g) {
#pragma unroll
    for (int c = 0; c < A::CPL; ++c) b[c] = *reinterpret_cast<const i32x4*>(lds + base + b_off(s, c, g));
  }

  // Software pipeline of one wave. The filter fragments of step s + ADEPTH are issued
  // before step s's MFMAs. B_RING: the B fragment of (step, M-tile) pair i + 2 is issued
  // before pair i's MFMAs, so two M-tiles of MFMAs hide each LDS read. B_ROLL: the B
  // fragment of M-tile mt for step s + 1 is issued right after the last MFMA of step s
  // that reads it, into the same registers. Scheduling barriers keep the compiler from
  // sinking the loads next to their uses.
  __device__ __forceinline__ static void run(AccV (&acc)[MT][NOT], const uint8_t* lds, const i32x4* __restrict__ wp,
                                             const int (&base)[MT], int lane) {
    const int g = lane >> 4;
    // A wave in its MFMA loop issues ahead of waves of the other work-group on the SIMD that
    // are staging or in an epilogue, whose VALU and memory instructions fill the MFMA gaps.
    __builtin_amdgcn_s_setprio(1);
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int ot = 0; ot < NOT; ++ot) acc[mt][ot] = AccV{};
    constexpr int NA = ADEPTH + 1;
    i32x4 a[NA][NOT][A::CPL];
#pragma unroll
    for (int d = 0; d < ADEPTH; ++d)
      if (d < NS) load_a(a[d], wp, d, lane);
    if constexpr (BMODE == B_RING) {
      constexpr int NP = NS * MT;  // pair i = (step i / MT, M-tile i % MT)
      i32x4 b[3][A::CPL];
      load_b(b[0], lds, base[0], 0, g);
      if (1 < NP) load_b(b[1], lds, base[1 % MT], 1 / MT, g);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s + ADEPTH < NS) load_a(a[(s + ADEPTH) % NA], wp, s + ADEPTH, lane);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const int i = s * MT + mt;
          if (i + 2 < NP) load_b(b[(i + 2) % 3], lds, base[(i + 2) % MT], (i + 2) / MT, g);
#pragma unroll
          for (int ot = 0; ot < NOT; ++ot) acc[mt][ot] = A::mma(a[s % NA][ot], b[i % 3], acc[mt][ot]);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else if constexpr (BMODE == B_ROLL) {
      i32x4 b[MT][A::CPL];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) load_b(b[mt], lds, base[mt], 0, g);
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s + ADEPTH < NS) load_a(a[(s + ADEPTH) % NA], wp, s + ADEPTH, lane);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
          for (int ot = 0; ot < NOT; ++ot) acc[mt][ot] = A::mma(a[s % NA][ot], b[mt], acc[mt][ot]);
          if (s + 1 < NS) load_b(b[mt], lds, base[mt], s + 1, g);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else {
      i32x4 b[MT][A::CPL];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s + ADEPTH < NS) load_a(a[(s + ADEPTH) % NA], wp, s + ADEPTH, lane);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) load_b(b[mt], lds, base[mt], s, g);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int ot = 0; ot < NOT; ++ot) acc[mt][ot] = A::mma(a[s % NA][ot], b[mt], acc[mt][ot]);
      }
    }
    __builtin_amdgcn_s_setprio(0);
  }
};

// The single-conv tile: M-tile mt of this wave is global M-tile index wave + NW*mt:
// OFDM symbol t = idx / (TW/16), subcarrier block cb = idx % (TW/16). Rows t >= T read
// the zero rows staged for them.
template <class A, int CIN, int COUT, int TW, int PITCH, int NW>
struct Gemm {
  static constexpr int MTOT = TMAX * (TW / 16);                  // M-tiles per tile (T = 14)
  static constexpr int MT = (MTOT + NW - 1) / NW;                // M-tiles per wave
  static constexpr int NOT = COUT / 16;
  using Core = GemmCore<A, CIN, COUT, TW + 2, PITCH, MT>;
  using AccV = typename A::AccV;

  __device__ __forceinline__ static void run(AccV (&acc)[MT][NOT], const uint8_t* lds, const i32x4* __restrict__ wp,
                                             int wave, int lane) {
    const int col = lane & 15;
    int base[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      int idx = wave + NW * mt;
      if (idx >= MTOT) idx = MTOT - 1;  // surplus tile of an uneven split: recompute a real one
      const int t = idx / (TW / 16), cb = idx - t * (TW / 16);
      base[mt] = (t * (TW + 2) + cb * 16 + col) * PITCH;
    }
    Core::run(acc, lds, wp, base, lane);
  }
};

// ---------------------------------------------------------------- block output
// Epilogue of a block's second conv for one RE: v holds conv + bias for this lane's EPL
// channels from c0 (lanes g = 0..3 of one column hold the RE's C channels). Adds the
// residual x (x_fn fills EPL values). On the main branch of a fused block (main_fused),
// keeps the pre-fusion output when save_o0 is set, multiplies (or with fuse_sum adds) in
// the stored support outputs of branches 1..K-1 (sup_fn(kk, values), kk < min(K, NSUP+1))
// and applies the per-RE LayerNorm over C (with norm_affine, BatchNorm with running statistics
// folded into gamma/beta: a per-channel affine); with sup_dst (Example II feedback) it also
// stores support output + fused activation to sup_dst[kk]. Then either the 1x1 LLR head
// (head) or a store of the block output to `out` (nullable). A plain block with the head
// stores its output to save_o0 when that is set (the backward's copy). LPR lanes (g =
// 0..LPR-1, 16 or 32 lanes apart) hold the C channels of one RE.
template <class A, int COUT, int EPL, int NSUP, class XFn, class SupFn, int LPR = 4>
__device__ __forceinline__ void finish_block(typename A::Acc (&v)[EPL], int64_t re, int c0, int g, bool main_fused,
                                             XFn x_fn, SupFn sup_fn, void* out, void* save_o0, bool head, int K,
                                             const float* gamma, const float* beta, float eps, const float* Wh,
                                             const float* bh, float* llr, int m, bool fuse_sum = false,
                                             void* const* sup_dst = nullptr, bool norm_affine = false) {
  using Acc = typename A::Acc;
  using Act = typename A::Act;
  {
    Acc x[EPL];
    x_fn(x);
#pragma unroll
    for (int i = 0; i < EPL; ++i) v[i] += x[i];
  }
  if (!main_fused) {
    if (head && save_o0) store_vals(reinterpret_cast<Act*>(save_o0) + re * COUT + c0, v, EPL, 1.f);
    if (!head && out) store_vals(reinterpret_cast<Act*>(out) + re * COUT + c0, v, EPL, 1.f);
  } else {  // product with the stored support outputs, then LayerNorm over C
    if (save_o0) store_vals(reinterpret_cast<Act*>(save_o0) + re * COUT + c0, v, EPL, 1.f);
#pragma unroll
    for (int kk = 1; kk <= NSUP; ++kk) {
      if (kk >= K) break;
      // two lanes per RE: one support tensor in registers at a time (the compiler would
      // otherwise issue every support's loads up front)
      if constexpr (LPR == 2) __builtin_amdgcn_sched_barrier(0);
      Acc sv[EPL];
      sup_fn(kk, sv);
      if (fuse_sum) {
#pragma unroll
        for (int i = 0; i < EPL; ++i) v[i] += sv[i];
      } else {
#pragma unroll
        for (int i = 0; i < EPL; ++i) v[i] *= sv[i];
      }
    }
    if (norm_affine) {
#pragma unroll
      for (int i = 0; i < EPL; ++i) v[i] = (Acc)gamma[c0 + i] * v[i] + (Acc)beta[c0 + i];
    } else {
      Acc s = 0;
#pragma unroll
      for (int i = 0; i < EPL; ++i) s += v[i];
      if (LPR == 4) s += __shfl_xor(s, 16);
      s += __shfl_xor(s, 32);
      const Acc mu = s * ((Acc)1 / (Acc)COUT);
      Acc q = 0;
#pragma unroll
      for (int i = 0; i < EPL; ++i) { const Acc d = v[i] - mu; q += d * d; }
      if (LPR == 4) q += __shfl_xor(q, 16);
      q += __shfl_xor(q, 32);
      const Acc rs = (Acc)1 / sqrtf((float)(q * ((Acc)1 / (Acc)COUT) + (Acc)eps));
#pragma unroll
      for (int i = 0; i < EPL; ++i) v[i] = (Acc)gamma[c0 + i] * (v[i] - mu) * rs + (Acc)beta[c0 + i];
    }
    if (sup_dst) {  // Example II: each support continues from its output plus the fused activation
#pragma unroll
      for (int kk = 1; kk <= NSUP; ++kk) {
        if (kk >= K) break;
        Acc sv[EPL];
        sup_fn(kk, sv);
#pragma unroll
        for (int i = 0; i < EPL; ++i) sv[i] += v[i];
        store_vals(reinterpret_cast<Act*>(sup_dst[kk]) + re * COUT + c0, sv, EPL, 1.f);
      }
    }
    if (!head && out) store_vals(reinterpret_cast<Act*>(out) + re * COUT + c0, v, EPL, 1.f);
  }
  if (head) {
    Acc part[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      part[j] = 0;
      if (j < m)
#pragma unroll
        for (int i = 0; i < EPL; ++i) part[j] += (Acc)Wh[j * COUT + c0 + i] * v[i];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (LPR == 4) part[j] += __shfl_xor(part[j], 16);
      part[j] += __shfl_xor(part[j], 32);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j < m && (j % LPR) == g) llr[re * m + j] = (float)(part[j] + (Acc)bh[j]);
  }
}

// ---------------------------------------------------------------- the kernel
// MODE 0: input layer            out = ReLU(conv(X) + b)
// MODE 1: first conv of a block  out = ReLU(s1 (conv(prologue(x)) + b1) + o1)   (or its max, calibration)
// MODE 2: second conv            out = x + conv(h) + b2; branch 0 of the last unfused block feeds the head
// MODE 4: second conv of the main net + fusion: O0 = x0 + conv(h0) + b2, P = O0 * prod_k sup_k
//         (the support outputs of this block, already stored), A = gamma LN(P) + beta -> out or head;
//         resid2 (training) also keeps O0
// MODE 5: backward through the second conv: dh = convT(dO); dz1 = dh [h > 0]; out = dc1 = s1 dz1;
//         partial sums of dz1 (h - o1) / s1, dz1, dc1 (-> ds1, do1, db1)
// MODE 6: backward through the first conv: dpre = convT(dc1); with z0 = s0 x + o0 (x for an MRB),
//         dz0 = dpre [z0 > 0]; out = dx = dO + s0 dz0 (dO + dz0 for an MRB), optionally times
//         [x > 0]; partial sums of dz0 x, dz0, out (-> ds0, do0, and db_in at the input layer)
template <class A, int MODE, int CIN, int COUT, int TW, int NW>
__global__ void __launch_bounds__(NW * 64, 2) conv3x3_kernel(ConvArgs args) {
  using Acc = typename A::Acc;
  using AccV = typename A::AccV;
  using Act = typename A::Act;
  using Hid = typename A::Hid;
  using InT = typename std::conditional<MODE == 0, float,
                                        typename std::conditional<(MODE == 2 || MODE == 4), Hid, Act>::type>::type;
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
  const int k0 = blockIdx.y + args.k_off;

  int prologue = 0;
  if (MODE == 1) prologue = args.pre_s[k0] ? 1 : 2;
  if (MODE == 0 && args.grid_rx > 0)
    stage_grid_tile<A, CIN, TW + 2, 1, PITCH, NT>(lds, reinterpret_cast<const float2*>(args.in[k0]), td, T,
                                                  args.grid_rx, args.in_qscale[k0]);
  else
    stage_tile<A, InT, CIN, TW + 2, 1, PITCH, NT>(lds, reinterpret_cast<const InT*>(args.in[k0]), td, T, prologue,
                                                  args.pre_s[k0], args.pre_o[k0], args.in_qscale[k0]);
  __syncthreads();
  // the input layer can run every branch from one staged tile (the features are shared)
  const int nb = (MODE == 0 && args.inner_branches > 1) ? args.inner_branches : 1;
  for (int kb = 0; kb < nb; ++kb) {
  const int k = k0 + kb;
  AccV acc[MT][NOT];
  // Backward through the second conv: the epilogue's mask operand h is loaded one M-tile ahead
  // as raw words into two alternating buffers and converted element by element where used, so
  // its latency overlaps the epilogue of the M-tile before; the first M-tile's is issued right
  // after the MFMA loop. (The same for x in mode 6 measured 5 % slower; x and dO together
  // did not fit the registers.)
  constexpr bool PREF = MODE == 5;
  using RawW = typename std::conditional<(EPL * sizeof(Act)) % 16 == 0, i32x4, uint2>::type;
  constexpr int NRW = PREF ? EPL * (int)sizeof(Act) / (int)sizeof(RawW) : 1;
  static_assert(!PREF || (EPL * sizeof(Act)) % sizeof(RawW) == 0, "epilogue operands fill whole words");
  RawW pra[2][NRW];
  auto epi_re = [&](int mt, int64_t& re) -> bool {
    const int idx = wave + NW * mt;
    const int t = idx / (TW / 16);
    const int f = td.f0 + (idx - t * (TW / 16)) * 16 + col;
    if (idx >= G::MTOT || t >= T || f >= td.F) return false;
    re = td.re_base + (int64_t)t * td.F + f;
    return true;
  };
  auto prefetch = [&](int mt) {
    int64_t re = 0;
    if (!epi_re(mt, re)) return;
    const RawW* a = reinterpret_cast<const RawW*>(reinterpret_cast<const Act*>(args.aux[k]) + re * COUT + c0);
#pragma unroll
    for (int w = 0; w < NRW; ++w) pra[mt & 1][w] = a[w];
  };
  // element i of a raw buffer, as the epilogue's type
  auto elem = [](const RawW* w, int i) -> Acc {
    const Act* e = reinterpret_cast<const Act*>(w);
    return (Acc)e[i];
  };
  G::run(acc, lds, reinterpret_cast<const i32x4*>(args.wpack[k]), wave, lane);
  if constexpr (PREF) prefetch(0);

  // per-lane epilogue parameters (this lane's EPL channels), loaded once
  float pb[EPL], pq[EPL];
  {
    const float* bias = args.bias[k];
    const float* ws = args.wscale[k];
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      pb[i] = bias[c0 + i];
      pq[i] = A::QUANT ? args.deq[k] * ws[c0 + i] : 1.0f;
    }
  }
  constexpr bool AFF = (MODE == 1 || MODE == 5 || MODE == 6);
  float ps1[AFF ? EPL : 1], po1[AFF ? EPL : 1];
  bool mrb = false;
  if constexpr (MODE == 1 || MODE == 5) {
#pragma unroll
    for (int i = 0; i < EPL; ++i) { ps1[i] = args.post_s[k][c0 + i]; po1[i] = args.post_o[k][c0 + i]; }
  } else if constexpr (MODE == 6) {
    mrb = args.pre_s[k] == nullptr;
#pragma unroll
    for (int i = 0; i < EPL; ++i) {
      ps1[i] = mrb ? 1.f : args.pre_s[k][c0 + i];
      po1[i] = mrb ? 0.f : args.pre_o[k][c0 + i];
    }
  }
  constexpr int NPART = MODE == 5 ? 3 : (MODE == 6 ? 3 : 1);
  float sums[NPART][(MODE == 5 || MODE == 6) ? EPL : 1];
#pragma unroll
  for (int q = 0; q < NPART; ++q)
#pragma unroll
    for (int i = 0; i < ((MODE == 5 || MODE == 6) ? EPL : 1); ++i) sums[q][i] = 0.f;
  unsigned amax_bits = 0;

#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    int64_t re = 0;
    const bool ok = epi_re(mt, re);
    if constexpr (PREF) {
      if (mt + 1 < MT) prefetch(mt + 1);
    }
    if (!ok) continue;
    Acc v[EPL];
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        Acc a = acc[mt][ot][i];
        if constexpr (A::QUANT) a = a * (Acc)pq[4 * ot + i];
        v[4 * ot + i] = (MODE == 5 || MODE == 6) ? a : a + (Acc)pb[4 * ot + i];  // input-gradient convs have no bias
      }
    if constexpr (MODE == 5) {  // dv = dh (the bias slot holds zeros for input-gradient convs)
#pragma unroll
      for (int i = 0; i < EPL; ++i) {
        const Acc h = elem(pra[mt & 1], i);
        const Acc dz = h > (Acc)0 ? v[i] : (Acc)0;
        const Acc dc = dz * (Acc)ps1[i];
        sums[0][i] += (float)(dz * (h - (Acc)po1[i]));  // divided by s1 once, after the sums
        sums[1][i] += (float)dz;
        sums[2][i] += (float)dc;
        v[i] = dc;
      }
      store_vals(reinterpret_cast<Act*>(args.out[k]) + re * COUT + c0, v, EPL, 1.f);
    } else if constexpr (MODE == 6) {
      Acc xv[EPL], dOv[EPL];
      load_vals(reinterpret_cast<const Act*>(args.aux[k]) + re * COUT + c0, xv, EPL);
      load_vals(reinterpret_cast<const Act*>(args.resid[k]) + re * COUT + c0, dOv, EPL);
#pragma unroll
      for (int i = 0; i < EPL; ++i) {
        const Acc x = xv[i], dO = dOv[i];
        const Acc z0 = (Acc)ps1[i] * x + (Acc)po1[i];
        const Acc dz = z0 > (Acc)0 ? v[i] : (Acc)0;
        Acc dx = dO + (Acc)ps1[i] * dz;
        if (args.mask_out && !(x > (Acc)0)) dx = (Acc)0;
        sums[0][i] += mrb ? 0.f : (float)(dz * x);
        sums[1][i] += mrb ? 0.f : (float)dz;
        sums[2][i] += (float)dx;
        v[i] = dx;
      }
      store_vals(reinterpret_cast<Act*>(args.out[k]) + re * COUT + c0, v, EPL, 1.f);
    } else if constexpr (MODE == 0) {
#pragma unroll
      for (int i = 0; i < EPL; ++i) v[i] = v[i] > (Acc)0 ? v[i] : (Acc)0;
      store_vals(reinterpret_cast<Act*>(args.out[k]) + re * COUT + c0, v, EPL, 1.f);
    } else if constexpr (MODE == 1) {
#pragma unroll
      for (int i = 0; i < EPL; ++i) {
        const Acc z = (Acc)ps1[i] * v[i] + (Acc)po1[i];
        v[i] = z > (Acc)0 ? z : (Acc)0;
      }
      if (args.amax) {
        float mx = 0.f;
#pragma unroll
        for (int i = 0; i < EPL; ++i) mx = fmaxf(mx, (float)v[i]);
        amax_bits = max(amax_bits, __float_as_uint(mx));
      } else {
        store_vals(reinterpret_cast<Hid*>(args.out[k]) + re * COUT + c0, v, EPL, args.out_qscale[k]);
      }
    } else {
      const bool head = MODE == 2 ? (args.llr && k == 0) : args.llr != nullptr;
      const Act* xr = reinterpret_cast<const Act*>(args.resid[k]) + re * COUT + c0;
      finish_block<A, COUT, EPL, KMAX_ARGS - 1>(
          v, re, c0, g, MODE == 4, [&](Acc* x) { load_vals(xr, x, EPL); },
          [&](int kk, Acc* sv) { load_vals(reinterpret_cast<const Act*>(args.sup[kk]) + re * COUT + c0, sv, EPL); },
          MODE == 2 ? args.out[k] : args.out[0], args.save_o0, head, args.K, args.gamma, args.beta, args.eps, args.Wh,
          args.bh, args.llr, args.m, args.fusion_sum != 0,
          (MODE == 4 && args.feedback) ? const_cast<void* const*>(args.sup) : nullptr, args.norm_affine != 0);
    }
  }
  if constexpr (MODE == 5 || MODE == 6) {
    // reduce the per-lane sums over the 16 lanes that own the same channels, then one
    // row of partial sums per wave (no atomics: the final reduction runs in a fixed order)
#pragma unroll
    for (int q = 0; q < NPART; ++q)
#pragma unroll
      for (int i = 0; i < EPL; ++i) {
        float t = sums[q][i];
        t += __shfl_xor(t, 1);
        t += __shfl_xor(t, 2);
        t += __shfl_xor(t, 4);
        t += __shfl_xor(t, 8);
        sums[q][i] = t;
      }
    if constexpr (MODE == 5) {  // ds1 = sum dz (h - o1) / s1: the conv output recovered from h
#pragma unroll
      for (int i = 0; i < EPL; ++i) sums[0][i] /= ps1[i];
    }
    if (col == 0) {
      float* row = args.part[k] + ((size_t)blockIdx.x * NW + wave) * NPART * COUT;
#pragma unroll
      for (int q = 0; q < NPART; ++q)
#pragma unroll
        for (int i = 0; i < EPL; ++i) row[q * COUT + c0 + i] = sums[q][i];
    }
  }
  if constexpr (MODE == 1) {
    if (args.amax) {  // calibration: one atomic per lane group
      for (int o = 32; o > 0; o >>= 1) amax_bits = max(amax_bits, (unsigned)__shfl_xor((int)amax_bits, o));
      if (lane == 0) atomicMax(args.amax + k, amax_bits);
    }
  }
  }  // branches
}

// ---------------------------------------------------------------- launch
// FP32 convs wider than 16 subcarriers also have a 16-wide build (forward modes only), for
// batches whose tiles cannot fill the GPU: on a single small slot each stage is a handful of
// work-groups, each doing a whole tile's GEMM, so narrower tiles cut the stage time.
template <class A, int CIN, int COUT>
constexpr int tile_w_narrow() {
  constexpr int TW = tile_w<A, CIN, COUT>();
  return (std::is_same<A, ArithF32>::value && TW > 16) ? 16 : TW;
}

template <class A, int MODE, int CIN, int COUT, int TW>
static hipError_t launch_tw(ConvArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  a.tw = TW;
  hipLaunchKernelGGL((conv3x3_kernel<A, MODE, CIN, COUT, TW, CONV_NW>), dim3(n_tiles, grid_y), dim3(CONV_NW * 64), 0,
                     s, a);
  return hipGetLastError();
}

template <class A, int MODE, int CIN, int COUT>
static hipError_t launch_one(ConvArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  constexpr int TW = tile_w<A, CIN, COUT>(), TWN = tile_w_narrow<A, CIN, COUT>();
  if constexpr (TWN != TW && MODE <= 4) {
    if (a.narrow) return launch_tw<A, MODE, CIN, COUT, TWN>(a, n_tiles, grid_y, s);
  }
  return launch_tw<A, MODE, CIN, COUT, TW>(a, n_tiles, grid_y, s);
}

template <class A, int CIN, int COUT>
static hipError_t launch_mode(int mode, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  if (CIN == COUT) {  // block convs
    switch (mode) {
      case 1: return launch_one<A, 1, CIN, COUT>(a, n_tiles, grid_y, s);
      case 2: return launch_one<A, 2, CIN, COUT>(a, n_tiles, grid_y, s);
      case 4: return launch_one<A, 4, CIN, COUT>(a, n_tiles, grid_y, s);
      case 5:
      case 6:
        if constexpr (sizeof(typename A::Op) == 1) return hipErrorInvalidValue;  // no FP8 training
        else return mode == 5 ? launch_one<A, 5, CIN, COUT>(a, n_tiles, grid_y, s)
                              : launch_one<A, 6, CIN, COUT>(a, n_tiles, grid_y, s);
    }
  }
  if (mode == 0) return launch_one<A, 0, CIN, COUT>(a, n_tiles, grid_y, s);
  return hipErrorInvalidValue;
}

// Channel pairs instantiated: input layers (C_in -> C) and blocks (C -> C) of the
// workloads (C_in 8/16/32, and 24 = 4 antennas + the variance channels; C 16/32/64/96).
#define CONET_PAIRS(X)                                                                                    \
  X(8, 16) X(8, 32) X(8, 64) X(16, 16) X(16, 32) X(16, 64) X(16, 96) X(24, 32) X(24, 64) X(32, 32) X(32, 96) \
  X(64, 64) X(96, 96)
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
int tile_width_narrow_dtype(int cin, int cout) {
#define CONET_TWN(CI, CO) \
  if (cin == CI && cout == CO) return tile_w_narrow<A, CI, CO>();
  if constexpr (sizeof(typename A::Op) == 1) {
    CONET_PAIRS_FP8(CONET_TWN)
  } else {
    CONET_PAIRS(CONET_TWN)
  }
#undef CONET_TWN
  return 0;
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
