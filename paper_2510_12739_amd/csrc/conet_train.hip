// Backward-pass and training kernels of CoNet-Rx (gfx950).
//
//  * wgrad_kernel: filter gradient of a 3x3 conv, dW[o][tap, ch] = sum over REs of
//    dOut[re][o] * In[re + tap][ch]. The reduction runs over REs, so both operands are
//    staged into LDS transposed (channel-major, RE-contiguous): an MFMA lane then reads
//    VEC consecutive REs of one channel with one 16-byte load. Taps shifted along the
//    subcarrier axis read two aligned 16-byte words and funnel-shift them. A thread
//    issues all of its staging loads of a tile before consuming any (one load in flight
//    at a time made the staging three times longer than the MFMAs). Each work-group
//    loops over a share of the tiles and writes one partial row; the rows are summed in
//    a fixed order by reduce_kernel (deterministic, no atomics).
//  * fuse_bwd_kernel: adjoint of the head, the per-RE LayerNorm (or BatchNorm by batch
//    statistics) and the K-way product, dO[k] = dP * prod_{j != k} O[j] (no division, so
//    exact zeros are handled).
//  * bn_stats_kernel, bn_finish_kernel: BatchNorm's per-channel batch mean and variance of
//    the product (two passes, fixed-order sums), the folded affine the fusion epilogue
//    applies, and the running statistics.
//  * bce_kernel, adam_kernel, repack_kernel, gather_kernel, reduce_kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "conet_common.h"
#include "conet_kernels.h"

namespace conet {

// ---------------------------------------------------------------- helpers
template <class T>
__device__ __forceinline__ float ldf(const T* p) { return (float)*p; }

__device__ __forceinline__ void to_elems(const i32x4& raw, float* v, const float*) {
  const float* f = reinterpret_cast<const float*>(&raw);
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = f[i];
}
__device__ __forceinline__ void to_elems(const i32x4& raw, float* v, const __bf16*) {
  const __bf16* b = reinterpret_cast<const __bf16*>(&raw);
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = (float)b[i];
}

template <class E>
__device__ __forceinline__ void st_elem(uint8_t* p, float v) {
  if constexpr (sizeof(E) == 4) *reinterpret_cast<float*>(p) = v;
  else *reinterpret_cast<__bf16*>(p) = f2bf(v);
}

// 16-byte window starting `s` elements into the 32 bytes lo:hi.
template <class E>
__device__ __forceinline__ i32x4 shift_window(const i32x4& lo, const i32x4& hi, int s) {
  const unsigned w[8] = {(unsigned)lo[0], (unsigned)lo[1], (unsigned)lo[2], (unsigned)lo[3],
                         (unsigned)hi[0], (unsigned)hi[1], (unsigned)hi[2], (unsigned)hi[3]};
  i32x4 r;
  if constexpr (sizeof(E) == 4) {
#pragma unroll
    for (int i = 0; i < 4; ++i) r[i] = (int)(s == 0 ? w[i] : (s == 1 ? w[i + 1] : w[i + 2]));
  } else {  // 2-byte elements: s = 1 is a 2-byte funnel shift, s = 2 a whole dword
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const unsigned a1 = __builtin_amdgcn_alignbyte(w[i + 1], w[i], 2);
      r[i] = (int)(s == 0 ? w[i] : (s == 1 ? a1 : w[i + 1]));
    }
  }
  return r;
}

// ---------------------------------------------------------------- wgrad
template <class A>
constexpr int wg_tw() { return 4 * A::VEC; }  // subcarriers per tile: one MFMA K step per OFDM symbol

// Eight waves, two per SIMD: while one waits on its LDS reads the other issues MFMAs (with four
// waves, one per SIMD, every fragment read stalled its wave's MFMAs). Wave w owns 16-wide
// (tap, channel) tiles kt = w, w + 8, ...: channel chunk w % (CIN/16) of taps w / (CIN/16) +
// j 8 / (CIN/16); each wave group's taps are compile-time constants of its own instantiation
// of the MFMA loop, so the tap offsets and the funnel shifts fold.
constexpr int WG_NW = 8;

// f(std::integral_constant<int, g>) for the runtime g in [0, N)
template <int N, class F>
__device__ __forceinline__ void dispatch_group(int g, F&& f) {
  if constexpr (N > 0) {
    if (g == N - 1) {
      f(std::integral_constant<int, N - 1>{});
      return;
    }
    dispatch_group<N - 1>(g, f);
  }
}

template <class A, class InT, int CIN, int COUT>
__global__ void __launch_bounds__(WG_NW * 64, 2) wgrad_kernel(WgradArgs args) {
  using E = typename A::Op;
  using Act = typename A::Act;
  using AccV = typename A::AccV;
  constexpr int VEC = A::VEC, TW = wg_tw<A>(), NW = WG_NW, NT = NW * 64;
  constexpr int ICOLS = TW + 8;                                    // TW+2 staged, room for shifted reads
  // channel strides (bytes): the rows plus 32 bytes, so that with the swizzle below the 16
  // channel rows of a fragment read start 16 x 8 banks apart on 64 banks (16 bytes left the
  // reads of the swizzled rows 2-way conflicted)
  constexpr int DS = TMAX * TW * (int)sizeof(E) + 32;              // dOut
  constexpr int IS = TROWS * ICOLS * (int)sizeof(E) + 32;          // In
  constexpr int NOT = COUT / 16, NKT = 9 * CIN / 16, KTW = (NKT + NW - 1) / NW;
  constexpr int CPT16 = CIN / 16, NG = NW / CPT16;                 // 16-channel chunks per tap, wave groups
  static_assert(NW % CPT16 == 0, "waves must cover whole taps");
  constexpr int EPD = 16 / (int)sizeof(Act), CPD = COUT / EPD;     // dOut: elements / chunks per RE
  constexpr int EPI = 16 / (int)sizeof(InT) < 4 ? 4 : 16 / (int)sizeof(InT), CPI = CIN / EPI;
  static_assert(NT % CPD == 0 && NT % CPI == 0 && CIN % 16 == 0 && COUT % 16 == 0, "shape");
  // Bank swizzle. A staging store instruction writes one channel of each of the wave's channel
  // chunks (8 lanes per RE); the chunks' channel rows lie a multiple of 32 banks apart, so
  // without it every chunk hit the same banks (an 8-way conflict). The 16-byte position block
  // of a channel row is XORed with the channel's chunk index (mod 8): stores spread over the
  // banks, and a fragment read (8 consecutive positions of one row) stays one aligned block.
  // Both tiles' rows hold a whole number of 8-block groups, so the XOR stays inside the row.
  static_assert((TMAX * TW) % (8 * VEC) == 0 && (TROWS * ICOLS) % (8 * VEC) == 0, "swizzle groups");
  auto swzD = [](int ch) { return ((ch / EPD) & 7) * VEC; };
  auto swzI = [](int ch) { return ((ch / EPI) & 7) * VEC; };
  extern __shared__ __attribute__((aligned(16))) uint8_t lds[];
  uint8_t* ldsD = lds;
  uint8_t* ldsI = lds + COUT * DS;

  const int k = blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 4, col = lane & 15;
  const Act* dout = reinterpret_cast<const Act*>(args.dout[k]);
  const InT* in = reinterpret_cast<const InT*>(args.in[k]);
  const int pro = args.prologue == 0 ? 0 : (args.pre_s[k] ? 1 : 2);
  const int ccD = tid % CPD, ccI = tid % CPI;
  // the prologue's per-channel affine sits in LDS behind the tiles and is read where it is
  // applied (in registers for the whole kernel it pushed the accumulators into scratch)
  float* pre_lds = reinterpret_cast<float*>(lds + COUT * DS + CIN * IS);
  if (pro == 1)
    for (int i = tid; i < 2 * CIN; i += NT) pre_lds[i] = i < CIN ? args.pre_s[k][i] : args.pre_o[k][i - CIN];
  AccV acc[NOT][KTW];
#pragma unroll
  for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
    for (int j = 0; j < KTW; ++j) acc[ot][j] = AccV{};
  float bsum[EPD];
#pragma unroll
  for (int i = 0; i < EPD; ++i) bsum[i] = 0.f;
  const int T = args.T;

  // 2-byte elements: the output-gradient tile of the work-group's next tile is loaded into
  // registers before the current tile's MFMAs (its latency then overlaps them)
  constexpr int NPD2 = TMAX * (TW / 2) * CPD, ND2 = sizeof(E) == 2 ? (NPD2 + NT - 1) / NT : 1;
  i32x4 pd0[ND2], pd1[ND2];
  auto load_dout_pairs = [&](int tile) {
    const int b = tile / args.tiles_per_slot;
    const int f0 = (tile - b * args.tiles_per_slot) * TW;
    const int64_t re_base = (int64_t)b * T * args.F;
#pragma unroll
    for (int u = 0; u < ND2; ++u) {
      const int idx = tid + u * NT;
      const int pp = idx / CPD;
      const int t = pp / (TW / 2), c = 2 * (pp - t * (TW / 2)), f = f0 + c;
      pd0[u] = i32x4{0, 0, 0, 0};
      pd1[u] = i32x4{0, 0, 0, 0};
      if (idx < NPD2 && t < T) {
        const Act* src = dout + (re_base + (int64_t)t * args.F + f) * COUT + ccD * EPD;
        if (f < args.F) pd0[u] = *reinterpret_cast<const i32x4*>(src);
        if (f + 1 < args.F) pd1[u] = *reinterpret_cast<const i32x4*>(src + COUT);
      }
    }
  };
  if constexpr (sizeof(E) == 2) {
    if ((int)blockIdx.x < args.n_tiles) load_dout_pairs(blockIdx.x);
  }

  for (int tile = blockIdx.x; tile < args.n_tiles; tile += gridDim.x) {
    const int b = tile / args.tiles_per_slot;
    const int f0 = (tile - b * args.tiles_per_slot) * TW;
    const int64_t re_base = (int64_t)b * T * args.F;
    __syncthreads();  // the previous tile's LDS reads are done
    // dOut tile [TMAX][TW] transposed to [o][t][c] and In halo tile [TROWS][TW+2] (prologue
    // inside the slot, zero padding outside) transposed to [ch][r][c]. A thread's 16-byte loads
    // are issued in batches before any of the batch is consumed, so their latencies overlap.
    // 2-byte elements: a lane loads one channel chunk of two adjacent subcarriers and writes
    // each channel's pair as one 4-byte word (2-byte stores of two lanes into one word conflict).
    if constexpr (sizeof(E) == 2) {
      constexpr int SB = 2;
#pragma unroll
      for (int u = 0; u < ND2; ++u) {
        const int idx = tid + u * NT;
        if (idx >= NPD2) break;
        const int pp = idx / CPD;
        const int t = pp / (TW / 2), c = 2 * (pp - t * (TW / 2));
        const int sw = swzD(ccD * EPD);
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const uint32_t a = (uint32_t)pd0[u][d], bb = (uint32_t)pd1[u][d];
          bsum[2 * d] += __uint_as_float(a << 16) + __uint_as_float(bb << 16);
          bsum[2 * d + 1] += __uint_as_float(a & 0xffff0000u) + __uint_as_float(bb & 0xffff0000u);
          uint8_t* dst = ldsD + (ccD * EPD + 2 * d) * DS + ((t * TW + c) ^ sw) * 2;
          *reinterpret_cast<uint32_t*>(dst) = (a & 0xffffu) | (bb << 16);
          *reinterpret_cast<uint32_t*>(dst + DS) = (a >> 16) | (bb & 0xffff0000u);
        }
      }
      constexpr int PPR = (TW + 2) / 2, NPI = TROWS * PPR * CPI, NI = (NPI + NT - 1) / NT;
      static_assert((TW + 2) % 2 == 0, "pairs per row");
#pragma unroll
      for (int u0 = 0; u0 < NI; u0 += SB) {
        i32x4 r0[SB], r1[SB];
        bool ok0[SB], ok1[SB];
#pragma unroll
        for (int u = u0; u < u0 + SB && u < NI; ++u) {
          const int idx = tid + u * NT;
          const int pp = idx / CPI;
          const int r = pp / PPR, c = 2 * (pp - r * PPR);
          const int t = r - 1, f = f0 + c - 1;
          const bool row_ok = idx < NPI && t >= 0 && t < T;
          ok0[u - u0] = row_ok && f >= 0 && f < args.F;
          ok1[u - u0] = row_ok && f + 1 >= 0 && f + 1 < args.F;
          r0[u - u0] = i32x4{0, 0, 0, 0};
          r1[u - u0] = i32x4{0, 0, 0, 0};
          const InT* src = in + (re_base + (int64_t)t * args.F + f) * CIN + ccI * EPI;
          if (ok0[u - u0]) r0[u - u0] = *reinterpret_cast<const i32x4*>(src);
          if (ok1[u - u0]) r1[u - u0] = *reinterpret_cast<const i32x4*>(src + CIN);
        }
#pragma unroll
        for (int u = u0; u < u0 + SB && u < NI; ++u) {
          const int idx = tid + u * NT;
          if (idx >= NPI) break;
          const int pp = idx / CPI;
          const int r = pp / PPR, c = 2 * (pp - r * PPR);
          float v0[EPI], v1[EPI];
          if constexpr (sizeof(InT) == 4) {
            const float* q0 = reinterpret_cast<const float*>(&r0[u - u0]);
            const float* q1 = reinterpret_cast<const float*>(&r1[u - u0]);
#pragma unroll
            for (int i = 0; i < EPI; ++i) { v0[i] = i < 4 ? q0[i] : 0.f; v1[i] = i < 4 ? q1[i] : 0.f; }
          } else {
            to_elems(r0[u - u0], v0, (const InT*)nullptr);
            to_elems(r1[u - u0], v1, (const InT*)nullptr);
          }
          if (pro == 1) {
#pragma unroll
            for (int i = 0; i < EPI; ++i) {
              const float sc = pre_lds[ccI * EPI + i], of = pre_lds[CIN + ccI * EPI + i];
              if (ok0[u - u0]) v0[i] = fmaxf(sc * v0[i] + of, 0.f);
              if (ok1[u - u0]) v1[i] = fmaxf(sc * v1[i] + of, 0.f);
            }
          } else if (pro == 2) {
#pragma unroll
            for (int i = 0; i < EPI; ++i) { v0[i] = fmaxf(v0[i], 0.f); v1[i] = fmaxf(v1[i], 0.f); }
          }  // outside the slot the raw values are zero: zero padding
          const int sw = swzI(ccI * EPI);
#pragma unroll
          for (int i = 0; i < EPI; ++i) {
            const uint32_t w = (uint32_t)__builtin_bit_cast(uint16_t, f2bf(v0[i])) |
                               ((uint32_t)__builtin_bit_cast(uint16_t, f2bf(v1[i])) << 16);
            *reinterpret_cast<uint32_t*>(ldsI + (ccI * EPI + i) * IS + ((r * ICOLS + c) ^ sw) * 2) = w;
          }
        }
      }
    } else {
      // dOut tile [TMAX][TW] transposed to [o][t][c]. A thread's 16-byte loads are issued in
      // batches of up to SB before any of the batch is consumed, so their latencies overlap.
      constexpr int SB = 4;
      constexpr int ND = (TMAX * TW * CPD + NT - 1) / NT;
#pragma unroll
      for (int u0 = 0; u0 < ND; u0 += SB) {
        i32x4 raw[SB];
#pragma unroll
        for (int u = u0; u < u0 + SB && u < ND; ++u) {
          const int idx = tid + u * NT;
          const int pos = idx / CPD;
          const int t = pos / TW, c = pos - t * TW, f = f0 + c;
          raw[u - u0] = i32x4{0, 0, 0, 0};
          if (idx < TMAX * TW * CPD && t < T && f < args.F)
            raw[u - u0] = *reinterpret_cast<const i32x4*>(dout + (re_base + (int64_t)t * args.F + f) * COUT + ccD * EPD);
        }
#pragma unroll
        for (int u = u0; u < u0 + SB && u < ND; ++u) {
          const int idx = tid + u * NT;
          if (idx >= TMAX * TW * CPD) break;
          const int pos = idx / CPD;
          const int t = pos / TW, c = pos - t * TW;
          float v[EPD];
          to_elems(raw[u - u0], v, (const Act*)nullptr);  // zero outside the slot
#pragma unroll
          for (int i = 0; i < EPD; ++i) {
            bsum[i] += v[i];
            st_elem<E>(ldsD + (ccD * EPD + i) * DS + ((t * TW + c) ^ swzD(ccD * EPD + i)) * (int)sizeof(E), v[i]);
          }
        }
      }
      // In halo tile [TROWS][TW+2] (prologue, then zero padding) transposed to [ch][r][c]
      constexpr int NI = (TROWS * (TW + 2) * CPI + NT - 1) / NT;
#pragma unroll
      for (int u0 = 0; u0 < NI; u0 += SB) {
        i32x4 raw[SB];
        bool ok[SB];
#pragma unroll
        for (int u = u0; u < u0 + SB && u < NI; ++u) {
          const int idx = tid + u * NT;
          const int pos = idx / CPI;
          const int r = pos / (TW + 2), c = pos - r * (TW + 2);
          const int t = r - 1, f = f0 + c - 1;
          ok[u - u0] = idx < TROWS * (TW + 2) * CPI && t >= 0 && t < T && f >= 0 && f < args.F;
          raw[u - u0] = i32x4{0, 0, 0, 0};
          if (ok[u - u0])
            raw[u - u0] = *reinterpret_cast<const i32x4*>(in + (re_base + (int64_t)t * args.F + f) * CIN + ccI * EPI);
        }
#pragma unroll
        for (int u = u0; u < u0 + SB && u < NI; ++u) {
          const int idx = tid + u * NT;
          if (idx >= TROWS * (TW + 2) * CPI) break;
          const int pos = idx / CPI;
          const int r = pos / (TW + 2), c = pos - r * (TW + 2);
          float v[EPI];
          if constexpr (sizeof(InT) == 4) {
            const float* q = reinterpret_cast<const float*>(&raw[u - u0]);
#pragma unroll
            for (int i = 0; i < EPI; ++i) v[i] = i < 4 ? q[i] : 0.f;
          } else {
            to_elems(raw[u - u0], v, (const InT*)nullptr);
          }
          if (ok[u - u0]) {
            if (pro == 1) {
#pragma unroll
              for (int i = 0; i < EPI; ++i)
                v[i] = fmaxf(pre_lds[ccI * EPI + i] * v[i] + pre_lds[CIN + ccI * EPI + i], 0.f);
            } else if (pro == 2) {
#pragma unroll
              for (int i = 0; i < EPI; ++i) v[i] = fmaxf(v[i], 0.f);
            }
          }  // else: zero padding (the raw value is zero)
#pragma unroll
          for (int i = 0; i < EPI; ++i)
            st_elem<E>(ldsI + (ccI * EPI + i) * IS + ((r * ICOLS + c) ^ swzI(ccI * EPI + i)) * (int)sizeof(E), v[i]);
        }
      }
    }
    __syncthreads();
    if constexpr (sizeof(E) == 2) {
      if (tile + (int)gridDim.x < args.n_tiles) load_dout_pairs(tile + gridDim.x);
    }
    const int ch = (wave % CPT16) * 16 + col;  // this lane's input channel in every tap
    const uint8_t* row = ldsI + ch * IS;
    const int sw = swzI(ch);
    dispatch_group<NG>(wave / CPT16, [&](auto group) {
      constexpr int G = decltype(group)::value;  // taps G, G + NG, G + 2 NG, ...
      for (int t = 0; t < T; ++t) {  // one MFMA K step per OFDM symbol: TW REs = 4 lane groups x VEC
        i32x4 af[NOT];
#pragma unroll
        for (int ot = 0; ot < NOT; ++ot)
          af[ot] = *reinterpret_cast<const i32x4*>(ldsD + (ot * 16 + col) * DS +
                                                    ((t * TW + g * VEC) ^ swzD(ot * 16 + col)) * (int)sizeof(E));
#pragma unroll
        for (int j = 0; j < KTW; ++j) {
          const int tap = G + NG * j;
          if (tap >= 9) break;
          const int dt = tap / 3, s = tap - dt * 3;
          const int p0 = (t + dt) * ICOLS + g * VEC;
          const i32x4 lo = *reinterpret_cast<const i32x4*>(row + (p0 ^ sw) * (int)sizeof(E));
          i32x4 bfr = lo;
          if (s != 0)
            bfr = shift_window<E>(lo, *reinterpret_cast<const i32x4*>(row + ((p0 + VEC) ^ sw) * (int)sizeof(E)), s);
#pragma unroll
          for (int ot = 0; ot < NOT; ++ot) acc[ot][j] = A::mma(&af[ot], &bfr, acc[ot][j]);
        }
      }
    });
  }
  // partial dW: D[o][k] in lane (col = k within the k-tile, rows 4g + i)
  float* pw = args.part_w[k] + (size_t)blockIdx.x * COUT * 9 * CIN;
#pragma unroll
  for (int j = 0; j < KTW; ++j) {
    const int kt = wave + NW * j;
    if (kt >= NKT) break;
#pragma unroll
    for (int ot = 0; ot < NOT; ++ot)
#pragma unroll
      for (int i = 0; i < 4; ++i) pw[(size_t)(ot * 16 + 4 * g + i) * 9 * CIN + kt * 16 + col] = acc[ot][j][i];
  }
  float* red = reinterpret_cast<float*>(lds);
  static_assert((size_t)NT * EPD * 4 <= (size_t)COUT * DS + (size_t)CIN * IS, "bias reduction exceeds the tiles' LDS");
  // partial db: threads with the same channel chunk hold disjoint RE sums
  __syncthreads();
#pragma unroll
  for (int i = 0; i < EPD; ++i) red[tid * EPD + i] = bsum[i];
  __syncthreads();
  if (tid < COUT) {
    const int cc = tid / EPD, i = tid - cc * EPD;
    float sum = 0.f;
    for (int t2 = cc; t2 < NT; t2 += CPD) sum += red[t2 * EPD + i];
    args.part_b[k][(size_t)blockIdx.x * COUT + tid] = sum;
  }
}

template <class A, class InT, int CIN, int COUT>
static hipError_t launch_wgrad_t(WgradArgs& a, int grid_y, hipStream_t s) {
  using E = typename A::Op;
  constexpr int TW = wg_tw<A>();
  constexpr size_t lds = (size_t)COUT * (TMAX * TW * sizeof(E) + 32) + (size_t)CIN * (TROWS * (TW + 8) * sizeof(E) + 32) +
                        2 * CIN * sizeof(float);
  static_assert(lds <= 160 * 1024, "wgrad tiles exceed LDS");
  a.tw = TW;
  const int grid = a.grid;
  if (grid < 1 || grid > 256 || grid > a.n_tiles) return hipErrorInvalidValue;
  hipError_t e = hipFuncSetAttribute((const void*)wgrad_kernel<A, InT, CIN, COUT>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((wgrad_kernel<A, InT, CIN, COUT>), dim3(grid, grid_y), dim3(WG_NW * 64), lds, s, a);
  return hipGetLastError();
}

int wgrad_tile_width(int dtype) { return dtype == DT_BF16 ? wg_tw<ArithBF16>() : wg_tw<ArithF32>(); }
int wgrad_grid(int n_tiles, int branches, int n_cu) {
  const int per = std::max(1, std::min(256, n_cu / std::max(1, branches)));
  return std::min(n_tiles, per);
}

hipError_t launch_wgrad(int dtype, bool in_f32, int cin, int cout, WgradArgs& a, int grid_y, hipStream_t s) {
#define CONET_WG(CI, CO)                                                                          \
  if (cin == CI && cout == CO) {                                                                  \
    if (dtype == DT_BF16)                                                                         \
      return in_f32 ? launch_wgrad_t<ArithBF16, float, CI, CO>(a, grid_y, s)                      \
                    : launch_wgrad_t<ArithBF16, __bf16, CI, CO>(a, grid_y, s);                    \
    if (dtype == DT_F32) return launch_wgrad_t<ArithF32, float, CI, CO>(a, grid_y, s);            \
  }
  CONET_WG(16, 32) CONET_WG(16, 64) CONET_WG(32, 32) CONET_WG(64, 64) CONET_WG(16, 16) CONET_WG(32, 64)
#undef CONET_WG
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- head / norm / product adjoint
// HEAD: this launch also back-propagates through the LLR head (the last block), accumulates
// the head bias gradient and stores the head's input A for head_wgrad_kernel, which forms the
// head weight gradient (held here, its m x C/4 accumulators per thread left one wave per
// SIMD: 2.7x the time of the other launches). BN: the norm is BatchNorm by batch statistics (per channel,
// over the batch) instead of the per-RE LayerNorm; both share
//   dP = (g - mean(g) - ahat mean(g ahat)) / sigma,  g = gamma dA,
// with the means over what the statistics were taken over. For BN those batch means are
// gamma dbeta / n and gamma dgamma / n, so pass 1 accumulates dgamma and dbeta and pass 2,
// after their reduction, forms dP.
template <class Act, int C, int KB, bool HEAD, bool BN>
__global__ void __launch_bounds__(256) fuse_bwd_kernel(FuseBwdArgs a) {
  constexpr int QC = C / 4;
  const int tid = threadIdx.x, q = tid & 3, wave = tid >> 6;
  const int c0 = q * QC;
  const int m = a.m;
  constexpr int NH = HEAD ? 8 : 1;  // head outputs accumulated by this launch
  constexpr int QB = BN ? QC : 1;
  float gam[QC], bet[QC], bet_acc[QC], gam_acc[QC], bh_acc[NH];
  float bmu[QB], brs[QB], bg1[QB], bg2[QB];
#pragma unroll
  for (int i = 0; i < QC; ++i) {
    gam[i] = a.fused ? a.gamma[c0 + i] : 1.f;
    bet[i] = a.fused ? a.beta[c0 + i] : 0.f;
    bet_acc[i] = 0.f;
    gam_acc[i] = 0.f;
  }
  if constexpr (BN) {
    const float inv_n = 1.f / (float)a.n_re;
#pragma unroll
    for (int i = 0; i < QC; ++i) {
      bmu[i] = a.bn_mu[c0 + i];
      brs[i] = a.bn_rs[c0 + i];
      bg1[i] = a.bn_pass == 2 ? gam[i] * a.bn_dbeta[c0 + i] * inv_n : 0.f;
      bg2[i] = a.bn_pass == 2 ? gam[i] * a.bn_dgamma[c0 + i] * inv_n : 0.f;
    }
  }
#pragma unroll
  for (int j = 0; j < NH; ++j) bh_acc[j] = 0.f;
  const float invC = 1.f / (float)C;
  const int64_t nthr = (int64_t)gridDim.x * 64;
  for (int64_t re = (int64_t)blockIdx.x * 64 + (tid >> 2); re < a.n_re; re += nthr) {
    float O[KB][QC], P[QC];
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      const Act* src = reinterpret_cast<const Act*>(a.O[kk]) + re * C + c0;
#pragma unroll
      for (int i = 0; i < QC; ++i) O[kk][i] = (float)src[i];
    }
#pragma unroll
    for (int i = 0; i < QC; ++i) {
      float p = O[0][i];
#pragma unroll
      for (int kk = 1; kk < KB; ++kk) p *= O[kk][i];
      P[i] = p;
    }
    float ah[QC], rs = 1.f;
    if constexpr (BN) {
#pragma unroll
      for (int i = 0; i < QC; ++i) ah[i] = (P[i] - bmu[i]) * brs[i];
    } else if (a.fused) {
      float s = 0.f;
#pragma unroll
      for (int i = 0; i < QC; ++i) s += P[i];
      s += __shfl_xor(s, 1);
      s += __shfl_xor(s, 2);
      const float mu = s * invC;
      float v = 0.f;
#pragma unroll
      for (int i = 0; i < QC; ++i) { const float d = P[i] - mu; v += d * d; }
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      rs = 1.f / sqrtf(v * invC + a.eps);
#pragma unroll
      for (int i = 0; i < QC; ++i) ah[i] = (P[i] - mu) * rs;
    }
    // gradient of the block's main activation
    float dA[QC];
    if constexpr (HEAD) {
      float dl[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) dl[j] = j < m ? a.dllr[re * m + j] : 0.f;
#pragma unroll
      for (int i = 0; i < QC; ++i) {
        float t = 0.f;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (j < m) t += a.Wh[j * C + c0 + i] * dl[j];
        dA[i] = t;
      }
      // head bias; the head's input A = gamma ahat + beta (fused) or O[0] (unfused) is stored
#pragma unroll
      for (int j = 0; j < NH; ++j)
        if (j < m && q == 0) bh_acc[j] += dl[j];
      if (a.a_out) {
        Act* dst = reinterpret_cast<Act*>(a.a_out) + re * C + c0;
#pragma unroll
        for (int i = 0; i < QC; ++i) dst[i] = (Act)(a.fused ? gam[i] * ah[i] + bet[i] : O[0][i]);
      }
    } else {
      const Act* src = reinterpret_cast<const Act*>(a.dA) + re * C + c0;
#pragma unroll
      for (int i = 0; i < QC; ++i) dA[i] = (float)src[i];
    }
    float dO[KB][QC];
    if constexpr (BN) {
#pragma unroll
      for (int i = 0; i < QC; ++i) {
        gam_acc[i] += dA[i] * ah[i];
        bet_acc[i] += dA[i];
      }
      if (a.bn_pass == 1) continue;  // the batch sums are not known yet: no dO in this pass
#pragma unroll
      for (int i = 0; i < QC; ++i) {
        const float dP = (gam[i] * dA[i] - bg1[i] - ah[i] * bg2[i]) * brs[i];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
          float others = 1.f;
#pragma unroll
          for (int jj = 0; jj < KB; ++jj)
            if (jj != kk) others *= O[jj][i];
          dO[kk][i] = dP * others;
        }
      }
    } else if (a.fused) {
      float g1 = 0.f, g2 = 0.f, gv[QC];
#pragma unroll
      for (int i = 0; i < QC; ++i) {
        gam_acc[i] += dA[i] * ah[i];
        bet_acc[i] += dA[i];
        gv[i] = gam[i] * dA[i];
        g1 += gv[i];
        g2 += gv[i] * ah[i];
      }
      g1 += __shfl_xor(g1, 1);
      g1 += __shfl_xor(g1, 2);
      g2 += __shfl_xor(g2, 1);
      g2 += __shfl_xor(g2, 2);
      g1 *= invC;
      g2 *= invC;
#pragma unroll
      for (int i = 0; i < QC; ++i) {
        const float dP = (gv[i] - g1 - ah[i] * g2) * rs;
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
          float others = 1.f;
#pragma unroll
          for (int jj = 0; jj < KB; ++jj)
            if (jj != kk) others *= O[jj][i];
          dO[kk][i] = dP * others;
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < QC; ++i) {
        dO[0][i] = dA[i];
#pragma unroll
        for (int kk = 1; kk < KB; ++kk) dO[kk][i] = 0.f;
      }
    }
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      if (!a.dO[kk]) continue;
      if (kk > 0 && a.dnext[kk]) {
        const Act* src = reinterpret_cast<const Act*>(a.dnext[kk]) + re * C + c0;
#pragma unroll
        for (int i = 0; i < QC; ++i) dO[kk][i] += (float)src[i];
      }
      Act* dst = reinterpret_cast<Act*>(a.dO[kk]) + re * C + c0;
#pragma unroll
      for (int i = 0; i < QC; ++i) dst[i] = (Act)dO[kk][i];
    }
  }
  // block partials: sum over the 16 REs of a wave sharing q, then over the 4 waves
  const int NP = 2 * C + 8 * C + 8;
  __shared__ float red[4][2 * C + 8 * C + 8];
  auto wsum = [&](float x) {
    x += __shfl_xor(x, 4);
    x += __shfl_xor(x, 8);
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    return x;
  };
#pragma unroll
  for (int i = 0; i < QC; ++i) {
    const float ga = wsum(gam_acc[i]), ba = wsum(bet_acc[i]);
    if ((tid & 63) < 4) { red[wave][c0 + i] = ga; red[wave][C + c0 + i] = ba; }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {  // head weight columns: zero here (head_wgrad_kernel writes them)
#pragma unroll
    for (int i = 0; i < QC; ++i)
      if ((tid & 63) < 4) red[wave][2 * C + j * C + c0 + i] = 0.f;
    const float bsum = j < NH ? wsum(bh_acc[j < NH ? j : 0]) : 0.f;
    if ((tid & 63) == 0) red[wave][10 * C + j] = bsum;
  }
  __syncthreads();
  if (!a.part) return;
  for (int i = tid; i < NP; i += 256)
    a.part[(size_t)blockIdx.x * NP + i] = red[0][i] + red[1][i] + red[2][i] + red[3][i];
}

hipError_t launch_fuse_bwd(int dtype, FuseBwdArgs& a, int grid, hipStream_t s) {
  if (a.bn_mu && (!a.fused || !a.bn_rs || (a.bn_pass != 1 && a.bn_pass != 2) ||
                  (a.bn_pass == 2 && (!a.bn_dgamma || !a.bn_dbeta))))
    return hipErrorInvalidValue;
#define CONET_FB(E, C_, K_, BN_)                                                                           \
  if (a.C == C_ && a.K == K_ && (a.bn_mu != nullptr) == BN_) {                                           \
    if (a.head) hipLaunchKernelGGL((fuse_bwd_kernel<E, C_, K_, true, BN_>), dim3(grid), dim3(256), 0, s, a); \
    else hipLaunchKernelGGL((fuse_bwd_kernel<E, C_, K_, false, BN_>), dim3(grid), dim3(256), 0, s, a);       \
    return hipGetLastError();                                                                            \
  }
#define CONET_FBC(E, C_, BN_) CONET_FB(E, C_, 1, BN_) CONET_FB(E, C_, 2, BN_) CONET_FB(E, C_, 3, BN_) CONET_FB(E, C_, 4, BN_)
  if (dtype == DT_BF16) {
    CONET_FBC(__bf16, 16, false) CONET_FBC(__bf16, 32, false) CONET_FBC(__bf16, 64, false)
    CONET_FBC(__bf16, 32, true) CONET_FBC(__bf16, 64, true)
  }
  if (dtype == DT_F32) {
    CONET_FBC(float, 16, false) CONET_FBC(float, 32, false) CONET_FBC(float, 64, false)
    CONET_FBC(float, 32, true) CONET_FBC(float, 64, true)
  }
#undef CONET_FBC
#undef CONET_FB
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- head weight gradient
// dWh[j][c] = sum over REs of dLLR[re][j] A[re][c], written into the head-weight columns of
// the fusion adjoint's partial rows (same grid, one row per work-group). A lane owns one
// 16-byte chunk of channels of one RE per step (a wave covers 64 / (C / EPV) REs), keeps
// m x EPV sums, and the lanes and waves of a work-group are summed in a fixed order.
template <class Act, int C>
__global__ void __launch_bounds__(256) head_wgrad_kernel(HeadWgradArgs a) {
  constexpr int EPV = 16 / (int)sizeof(Act), CPR = C / EPV, RPW = 64 / CPR;
  static_assert(C % EPV == 0 && 64 % CPR == 0, "shape");
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int cc = lane % CPR, rsub = lane / CPR;
  const int m = a.m;
  float acc[8][EPV];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int e = 0; e < EPV; ++e) acc[j][e] = 0.f;
  const int64_t step = (int64_t)gridDim.x * 4 * RPW;
  for (int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * RPW; r0 < a.n_re; r0 += step) {
    const int64_t re = r0 + rsub;
    if (re >= a.n_re) continue;
    const i32x4 raw = *reinterpret_cast<const i32x4*>(reinterpret_cast<const Act*>(a.A) + re * C + cc * EPV);
    const Act* av = reinterpret_cast<const Act*>(&raw);
    float dl[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) dl[j] = j < m ? a.dllr[re * m + j] : 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int e = 0; e < EPV; ++e) acc[j][e] = fmaf(dl[j], (float)av[e], acc[j][e]);
  }
  __shared__ float red[4][8 * C];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int e = 0; e < EPV; ++e) {
      float x = acc[j][e];
#pragma unroll
      for (int o = CPR; o < 64; o <<= 1) x += __shfl_xor(x, o);
      if (rsub == 0) red[wave][j * C + cc * EPV + e] = x;
    }
  __syncthreads();
  for (int i = tid; i < m * C; i += 256)
    a.part[(size_t)blockIdx.x * a.ld + a.col0 + i] = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
}

hipError_t launch_head_wgrad(int dtype, int C, HeadWgradArgs& a, int grid, hipStream_t s) {
  if (a.m < 1 || a.m > 8 || a.n_re <= 0) return hipErrorInvalidValue;
#define CONET_HW(E, C_) \
  if (C == C_) { hipLaunchKernelGGL((head_wgrad_kernel<E, C_>), dim3(grid), dim3(256), 0, s, a); return hipGetLastError(); }
  if (dtype == DT_BF16) { CONET_HW(__bf16, 16) CONET_HW(__bf16, 32) CONET_HW(__bf16, 64) }
  if (dtype == DT_F32) { CONET_HW(float, 16) CONET_HW(float, 32) CONET_HW(float, 64) }
#undef CONET_HW
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- BatchNorm statistics
// Threads as in the adjoint above: four per RE, each over C/4 consecutive channels; the
// product is formed in the order the fusion epilogue forms it, so both see the same P.
template <class Act, int C>
__global__ void __launch_bounds__(256) bn_stats_kernel(BnStatsArgs a) {
  constexpr int QC = C / 4;
  const int tid = threadIdx.x, q = tid & 3, wave = tid >> 6, c0 = q * QC;
  float mu[QC], acc[QC];
#pragma unroll
  for (int i = 0; i < QC; ++i) {
    mu[i] = a.pass ? a.mean[c0 + i] : 0.f;
    acc[i] = 0.f;
  }
  const int64_t nthr = (int64_t)gridDim.x * 64;
  for (int64_t re = (int64_t)blockIdx.x * 64 + (tid >> 2); re < a.n_re; re += nthr) {
    float P[QC];
    const Act* src = reinterpret_cast<const Act*>(a.main) + re * C + c0;
#pragma unroll
    for (int i = 0; i < QC; ++i) P[i] = (float)src[i];
    for (int k = 1; k < a.K; ++k) {
      const Act* sk = reinterpret_cast<const Act*>(a.sup[k]) + re * C + c0;
#pragma unroll
      for (int i = 0; i < QC; ++i) P[i] *= (float)sk[i];
    }
#pragma unroll
    for (int i = 0; i < QC; ++i) {
      const float d = P[i] - mu[i];
      acc[i] = a.pass ? fmaf(d, d, acc[i]) : acc[i] + P[i];
    }
  }
  __shared__ float red[4][C];
#pragma unroll
  for (int i = 0; i < QC; ++i) {
    float x = acc[i];
    x += __shfl_xor(x, 4);
    x += __shfl_xor(x, 8);
    x += __shfl_xor(x, 16);
    x += __shfl_xor(x, 32);
    if ((tid & 63) < 4) red[wave][c0 + i] = x;
  }
  __syncthreads();
  for (int c = tid; c < C; c += 256)
    a.part[(size_t)blockIdx.x * C + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

// One work-group: four threads per channel sum every fourth partial, then combine.
__global__ void __launch_bounds__(256) bn_finish_kernel(BnFinishArgs a) {
  const int tid = threadIdx.x, c = tid >> 2, j = tid & 3;
  float s = 0.f;
  if (c < a.C)
    for (int g = j; g < a.groups; g += 4) s += a.part[(size_t)g * a.C + c];
  s += __shfl_xor(s, 1);
  s += __shfl_xor(s, 2);
  if (c >= a.C || j != 0) return;
  const float n = (float)a.n_re;
  if (a.pass == 0) {
    a.mean[c] = s / n;
    return;
  }
  const float var = s / n;
  const float rs = 1.f / sqrtf(var + a.eps);
  const float sc = a.gamma[c] * rs;
  a.rs[c] = rs;
  a.scale[c] = sc;
  a.shift[c] = a.beta[c] - a.mean[c] * sc;
  if (a.running_mean) {
    const float unbiased = a.n_re > 1 ? var * (n / (n - 1.f)) : var;
    a.running_mean[c] = (1.f - a.momentum) * a.running_mean[c] + a.momentum * a.mean[c];
    a.running_var[c] = (1.f - a.momentum) * a.running_var[c] + a.momentum * unbiased;
  }
}

int bn_stats_grid(int64_t n_re) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n_re + 63) / 64)); }

hipError_t launch_bn_stats(int dtype, BnStatsArgs& a, int grid, hipStream_t s) {
  if (a.n_re <= 0 || a.K < 1 || a.K > KMAX_ARGS) return hipErrorInvalidValue;
  if (dtype == DT_BF16 && a.C == 64) hipLaunchKernelGGL((bn_stats_kernel<__bf16, 64>), dim3(grid), dim3(256), 0, s, a);
  else if (dtype == DT_BF16 && a.C == 32) hipLaunchKernelGGL((bn_stats_kernel<__bf16, 32>), dim3(grid), dim3(256), 0, s, a);
  else if (dtype == DT_F32 && a.C == 64) hipLaunchKernelGGL((bn_stats_kernel<float, 64>), dim3(grid), dim3(256), 0, s, a);
  else if (dtype == DT_F32 && a.C == 32) hipLaunchKernelGGL((bn_stats_kernel<float, 32>), dim3(grid), dim3(256), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_bn_finish(BnFinishArgs& a, hipStream_t s) {
  if (a.C < 1 || a.C > 64 || a.groups < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bn_finish_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- reductions
// Stage 1: block (column block of 64, row chunk, segment); 256 threads = 64 columns x 4
// row lanes, each lane sums every 4th row of the chunk, then the 4 lanes are combined.
__global__ void __launch_bounds__(256) reduce_stage1(const ReduceSeg* segs) {
  const ReduceSeg sg = segs[blockIdx.z];
  const int chunks = (sg.rows + REDUCE_CHUNK - 1) / REDUCE_CHUNK;
  const int ck = blockIdx.y;
  if (ck >= chunks) return;
  const int j = blockIdx.x * 64 + (threadIdx.x & 63), rl = threadIdx.x >> 6;
  const int r0 = ck * REDUCE_CHUNK, r1 = min(sg.rows, r0 + REDUCE_CHUNK);
  float a = 0.f;
  if (j < sg.cols)
    for (int r = r0 + rl; r < r1; r += 4) a += sg.src[(size_t)r * sg.ld + j];
  __shared__ float red[4][64];
  red[rl][threadIdx.x & 63] = a;
  __syncthreads();
  if (rl == 0 && j < sg.cols)
    sg.tmp[(size_t)ck * sg.cols + j] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__global__ void __launch_bounds__(256) reduce_stage2(const ReduceSeg* segs) {
  const ReduceSeg sg = segs[blockIdx.y];
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= sg.cols) return;
  const int chunks = (sg.rows + REDUCE_CHUNK - 1) / REDUCE_CHUNK;
  float s = 0.f;
  for (int c = 0; c < chunks; ++c) s += sg.tmp[(size_t)c * sg.cols + j];
  int dj = j;
  if (sg.map == 1) {
    const int kk = 9 * sg.cin;
    const int o = j / kk, rem = j - o * kk, tap = rem / sg.cin, ch = rem - tap * sg.cin;
    dj = (o * sg.cin + ch) * 9 + tap;
  }
  sg.dst[dj] = s;
}

hipError_t launch_reduce(const ReduceSeg* segs_dev, int n_segs, int max_cols, int max_chunks, hipStream_t s) {
  if (n_segs == 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_stage1, dim3((max_cols + 63) / 64, max_chunks, n_segs), dim3(256), 0, s, segs_dev);
  hipLaunchKernelGGL(reduce_stage2, dim3((max_cols + 255) / 256, n_segs), dim3(256), 0, s, segs_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------- loss and optimiser
// Bitwise BCE with logits over data REs: loss partial sums per block, d loss / d LLR.
__global__ void __launch_bounds__(256) bce_kernel(const float* llr, const uint8_t* bits, const uint8_t* dmask,
                                                  int64_t n, int T, int F, int m, float inv_count, float* dllr,
                                                  float* part) {
  float acc = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t re = i / m;
    const int f = (int)(re % F), t = (int)((re / F) % T);
    const float z = llr[i], b = (float)bits[i];
    const bool data = dmask[t * F + f] != 0;
    const float l = fmaxf(z, 0.f) - z * b + log1pf(expf(-fabsf(z)));
    const float sg = 1.f / (1.f + expf(-z));
    dllr[i] = data ? (sg - b) * inv_count : 0.f;
    if (data) acc += l;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  __shared__ float w[4];
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (w[0] + w[1] + w[2] + w[3]) * inv_count;
}

hipError_t launch_bce(const float* llr, const uint8_t* bits, const uint8_t* dmask, int64_t n_re, int T, int F, int m,
                      float inv_count, float* dllr, float* part, int grid, hipStream_t s) {
  hipLaunchKernelGGL(bce_kernel, dim3(grid), dim3(256), 0, s, llr, bits, dmask, n_re * m, T, F, m, inv_count, dllr, part);
  return hipGetLastError();
}

// Adam on the FP32 master copy (bias-corrected moments).
__global__ void __launch_bounds__(256) adam_kernel(float* w, const float* g, float* mo, float* ve, int64_t n, float lr,
                                                   float b1, float b2, float eps, float bc1, float bc2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float m1 = b1 * mo[i] + (1.f - b1) * gi;
    const float v1 = b2 * ve[i] + (1.f - b2) * gi * gi;
    mo[i] = m1;
    ve[i] = v1;
    w[i] -= lr * (m1 / bc1) / (sqrtf(v1 / bc2) + eps);
  }
}

hipError_t launch_adam(float* w, const float* g, float* mo, float* ve, int64_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t s) {
  const int grid = (int)((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048);
  hipLaunchKernelGGL(adam_kernel, dim3(grid), dim3(256), 0, s, w, g, mo, ve, n, lr, b1, b2, eps, bc1, bc2);
  return hipGetLastError();
}

// Fragment-ordered filters regenerated from the FP32 master: dst[e] = W[map[e]] (0 where map < 0).
__global__ void __launch_bounds__(256) repack_kernel(const float* master, const int32_t* map, void* dst, int64_t n,
                                                     int dtype) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int32_t j = map[i];
    const float v = j >= 0 ? master[j] : 0.f;
    if (dtype == DT_BF16) reinterpret_cast<__bf16*>(dst)[i] = f2bf(v);
    else reinterpret_cast<float*>(dst)[i] = v;
  }
}

hipError_t launch_repack(const float* master, const int32_t* map, void* dst, int64_t n, int dtype, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int grid = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(repack_kernel, dim3(grid), dim3(256), 0, s, master, map, dst, n, dtype);
  return hipGetLastError();
}

// Per-channel vectors regenerated from the master: dst[i] = W[map[i]] where map >= 0.
__global__ void __launch_bounds__(256) gather_kernel(const float* master, const int32_t* map, float* dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int32_t j = map[i];
    if (j >= 0) dst[i] = master[j];
  }
}

hipError_t launch_gather(const float* master, const int32_t* map, float* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int grid = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  hipLaunchKernelGGL(gather_kernel, dim3(grid), dim3(256), 0, s, master, map, dst, n);
  return hipGetLastError();
}

// Sum of n floats into *out (one work-group, fixed order).
__global__ void __launch_bounds__(256) sum_kernel(const float* x, int n, float* out) {
  __shared__ float r[256];
  float a = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) a += x[i];
  r[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int i = 0; i < 256; ++i) t += r[i];
    *out = t;
  }
}

hipError_t launch_sum(const float* x, int n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, x, n, out);
  return hipGetLastError();
}

}  // namespace conet
