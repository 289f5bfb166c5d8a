// Launch sequence of the CoNet-Rx forward pass and the FP8 calibration pass.
//
// Stage order (the paper's sequential depth is 2L + 2 conv layers; the head is fused
// into the last one):
//   input layer of all K branches (one launch, grid.y = branch)
//   for each block l: first conv of every branch (grid.y = branch); then, with fusion
//   after block l, the second conv of the support branches (their outputs are stored)
//   followed by the second conv of the main branch, whose epilogue multiplies in the
//   stored support outputs and applies the LayerNorm (and the head after the last
//   block); without fusion, the second conv of every branch in one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <cmath>
#include <vector>

#include "conet_model.h"

namespace conet {

// ---------------------------------------------------------------- amax reduction
// max over REs and channels of |prologue(x)|, prologue 0: x, 1: ReLU(s0 x + o0), 2: ReLU(x)
template <class T>
__global__ void __launch_bounds__(256) amax_kernel(const T* __restrict__ x, int64_t n, int C, const float* s0,
                                                   const float* o0, int prologue, unsigned* out) {
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    float v = (float)x[i];
    if (prologue == 1) { const int c = (int)(i % C); v = fmaxf(s0[c] * v + o0[c], 0.f); }
    else if (prologue == 2) v = fmaxf(v, 0.f);
    m = fmaxf(m, fabsf(v));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

hipError_t launch_amax(const void* x, int elem_bytes, int64_t n_re, int C, const float* s0, const float* o0,
                       int prologue, unsigned* out, hipStream_t s) {
  const int64_t n = n_re * C;
  const int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
  if (blocks <= 0) return hipSuccess;
  if (elem_bytes == 4)
    hipLaunchKernelGGL(amax_kernel<float>, dim3(blocks), dim3(256), 0, s, (const float*)x, n, C, s0, o0, prologue, out);
  else
    hipLaunchKernelGGL(amax_kernel<__bf16>, dim3(blocks), dim3(256), 0, s, (const __bf16*)x, n, C, s0, o0, prologue, out);
  return hipGetLastError();
}

static int scale_index(int K, int L, int k, int l, int which) { (void)K; return 1 + 2 * (k * L + l) + which; }

// ---------------------------------------------------------------- fused blocks
// Schedules the blocks as fused launches (both convs of a block per work-group). Per block
// l: without fusion after it, one launch over the branches; with fusion, the support
// branches, then the main branch with the fusion epilogue (product or sum, LayerNorm and,
// after the last block, the head). The main branch of block l and the support branches of
// block l + 1 read disjoint inputs (the supports' outputs of block l, and those only), so
// unless Example II feedback makes supports depend on the main branch they share one
// launch (BLOCK_PAIR): 2 launches per fused block become one, which halves the dependent
// launches of a forward. Stage marks stay three per block: (a) a block without fusion,
// (b) support branches (paired with the previous block's main branch when paired),
// (c) a main branch launched alone (the last block's, or one that could not be paired).
struct FusedScheduler {
  conet_model* M;
  const Geometry& geo;
  int n_tiles;
  const TileDesc* tiles;
  int tw;
  int wclass;  // the width class of tw (TW_WIDE, TW_NARROW, TW_NARROW3)
  float* llr;
  hipStream_t s;
  int32_t* units;  // per-stage conv-branch units (two per fused branch block), or null
  bool pending = false;  // a main-branch launch of the previous block not issued yet
  BlockArgs main_args = {};

  // geometry + shared fields
  void base(BlockArgs& b) const {
    const conet_config& c = M->cfg;
    b.T = geo.T;
    b.F = geo.uniform ? geo.F : 0;
    b.tiles_per_slot = geo.uniform ? (geo.F + tw - 1) / tw : 0;
    b.tiles = geo.uniform ? nullptr : tiles;
    b.K = c.branches;
    b.eps = c.ln_eps;
    b.m = c.bits_per_symbol;
  }
  // branch k's block-l parameters, input x and output out into slot k of b
  void branch(BlockArgs& b, int k, int l, bool mrb, const void* x, void* out) const {
    const conet_config& c = M->cfg;
    const Layout& lay = M->lay;
    const int K = c.branches, L = c.blocks, C = c.channels;
    uint8_t* ws = M->ws;
    const float* vec = reinterpret_cast<const float*>(ws + lay.vec);
    const std::vector<float>& sc = M->act_scales;
    const float* vb = vec + lay.v_blk[k][l];
    b.x[k] = x;
    b.out[k] = out;
    b.pre_s[k] = mrb ? nullptr : vb + 0 * C;
    b.pre_o[k] = mrb ? nullptr : vb + 1 * C;
    b.b1[k] = vb + 2 * C;
    b.post_s[k] = vb + 3 * C;
    b.post_o[k] = vb + 4 * C;
    b.b2[k] = vb + 5 * C;
    b.ws1[k] = vb + 6 * C;
    b.ws2[k] = vb + 7 * C;
    b.w1[k] = ws + lay.w1f[k][l];
    b.w2[k] = ws + lay.w2f[k][l];
    const float s1 = sc[scale_index(K, L, k, l, 0)], s2 = sc[scale_index(K, L, k, l, 1)];
    b.q1[k] = 1.0f / s1;
    b.deq1[k] = s1;
    b.q2[k] = 1.0f / s2;
    b.deq2[k] = s2;
  }
  conet_status launch(int kind, BlockArgs& b, int grid_y, int stage, int n_blocks, const char* what) {
    const hipError_t e = launch_block(M->cfg.dtype, kind, wclass, M->cfg.channels, b, n_tiles, grid_y, s);
    if (e != hipSuccess) return hip_fail(e, what);
    if (units) units[stage] += 2 * n_blocks;
    return CONET_OK;
  }
  conet_status flush(int stage) {
    if (!pending) return CONET_OK;
    pending = false;
    return launch(BLOCK_MAIN, main_args, 1, stage, 1, "fused main block launch");
  }

  // Block l of every branch: in(k) / out(k) are the block's input and output buffers.
  // Training forwards also pass hid(k) (where h is saved) and o0 (the main branch's output
  // before the fusion, or branch 0's before the head); both null otherwise.
  template <class InFn, class OutFn, class HidFn, class MarkFn>
  conet_status block(int l, bool fuse, bool fused_prev, bool last, int Kl, InFn in, OutFn out, HidFn hid, void* o0,
                     MarkFn& mark) {
    const conet_config& c = M->cfg;
    const Layout& lay = M->lay;
    const int K = c.branches;
    const float* vec = reinterpret_cast<const float*>(M->ws + lay.vec);
    const int sa = 1 + 3 * l, sb = 2 + 3 * l, sc_ = 3 + 3 * l;
    conet_status st = CONET_OK;
    hipError_t e = mark();  // (a)
    if (e != hipSuccess) return hip_fail(e, "event record");
    if (!fuse) {
      st = flush(sa);
      if (st != CONET_OK) return st;
      const int nk = last ? 1 : Kl;  // after the last block only branch 0 feeds the head
      BlockArgs b = {};
      base(b);
      for (int k = 0; k < nk; ++k) {
        branch(b, k, l, k == 0 && fused_prev, in(k), last ? nullptr : out(k));
        b.hid_out[k] = hid(k);
      }
      b.llr = last ? llr : nullptr;
      b.save_o0 = last ? o0 : nullptr;  // kept where the head reads branch 0's output
      b.Wh = vec + lay.v_wh;
      b.bh = vec + lay.v_bh;
      st = launch(BLOCK_PLAIN, b, nk, sa, nk, "fused block launch");
      if (st != CONET_OK) return st;
      e = mark();  // (b)
      if (e == hipSuccess) e = mark();  // (c)
      return e == hipSuccess ? CONET_OK : hip_fail(e, "event record");
    }
    e = mark();  // (b)
    if (e != hipSuccess) return hip_fail(e, "event record");
    if (K > 1) {
      if (pending && !c.feedback) {  // previous main branch + these supports in one launch
        BlockArgs b = main_args;
        for (int k = 1; k < K; ++k) {
          branch(b, k, l, false, in(k), out(k));
          b.hid_out[k] = hid(k);
        }
        pending = false;
        st = launch(BLOCK_PAIR, b, K, sb, K, "paired block launch");
      } else {
        st = flush(sb);
        if (st != CONET_OK) return st;
        BlockArgs b = {};
        base(b);
        for (int k = 1; k < K; ++k) {
          branch(b, k, l, false, in(k), out(k));
          b.hid_out[k] = hid(k);
        }
        b.k_off = 1;
        st = launch(BLOCK_PLAIN, b, K - 1, sb, K - 1, "fused support block launch");
      }
    } else {
      st = flush(sb);
    }
    if (st != CONET_OK) return st;
    // the main branch of this block: run now after the last block, else deferred
    BlockArgs m = {};
    base(m);
    branch(m, 0, l, fused_prev, in(0), last ? nullptr : out(0));
    m.hid_out[0] = hid(0);
    m.save_o0 = o0;
    for (int k = 1; k < K; ++k) m.sup[k] = out(k);
    m.gamma = vec + lay.v_gamma[l];
    m.beta = vec + lay.v_beta[l];
    m.Wh = vec + lay.v_wh;
    m.bh = vec + lay.v_bh;
    m.llr = last ? llr : nullptr;
    m.fusion_sum = c.fusion_op == CONET_FUSE_SUM;
    m.norm_affine = c.norm == CONET_NORM_BN;
    m.feedback = c.feedback && !last;  // the supports' outputs are not read after the last block
    e = mark();  // (c)
    if (e != hipSuccess) return hip_fail(e, "event record");
    if (last) return launch(BLOCK_MAIN, m, 1, sc_, 1, "fused main block launch");
    main_args = m;
    pending = true;
    return CONET_OK;
  }
};

// ---------------------------------------------------------------- forward
conet_status run_forward(conet_model* M, const Arena& ar, const float* x, const Geometry& geo, float* llr,
                         hipStream_t s, std::vector<float>* calib, hipEvent_t* events, bool save, int32_t* units) {
  const conet_config& c = M->cfg;
  const Layout& lay = M->lay;
  const int K = c.branches, L = c.blocks, C = c.channels, Ci = c.in_channels, dt = c.dtype;
  uint8_t* ws = M->ws;
  float* vec = reinterpret_cast<float*>(ws + lay.vec);
  std::vector<float>& sc = M->act_scales;
  // a uniform inference batch whose block tiles cannot give every CU a work-group runs the
  // convs on their narrow tiles (FP32: 16 subcarriers; the same arithmetic per RE)
  const bool narrow = geo.uniform && !calib && !save &&
                      (int64_t)geo.B * ((geo.F + conv_tile_width(dt, C, C) - 1) / conv_tile_width(dt, C, C)) * K <
                          (int64_t)M->n_cu;
  const int tw_in = narrow ? conv_tile_width_narrow(dt, Ci, C) : conv_tile_width(dt, Ci, C);
  const int tw_blk = narrow ? conv_tile_width_narrow(dt, C, C) : conv_tile_width(dt, C, C);
  // Inference runs each block as one fused launch when a fused kernel exists for
  // (dtype, C); calibration and the training forward (which stores h) use two convs.
  const bool ds = c.block_type == CONET_BLOCK_SEPARABLE;
  const bool concat = c.fusion_op == CONET_FUSE_CONCAT;
  const int Ls = support_depth(c);
  // a training model with BatchNorm normalises by the batch's own statistics: at its fused
  // levels the block launches store every branch output, and the fusion epilogue runs as a
  // pass of its own after the per-channel statistics of the product (bn_epilogue below)
  const bool bn_batch = c.train && c.norm == CONET_NORM_BN;
  int tw_fb = (calib || ds) ? 0 : block_tile_width(dt, C, K, TW_WIDE, c.train != 0);
  // a batch whose wide tiles cannot fill the GPU once (a slot, a serving batch) runs on
  // narrow tiles: more, shorter work-groups per launch; if its paired launches (K branches
  // per tile) would then hold more than two work-groups per CU, on the build for three
  int wclass = TW_WIDE;
  if (tw_fb) {
    auto tiles_at = [&](int tw) {
      int64_t n = 0;
      if (geo.uniform) {
        n = (int64_t)geo.B * ((geo.F + tw - 1) / tw);
      } else {
        for (int sl = 0; sl < geo.n_slots; ++sl) n += (geo.F_host[sl] + tw - 1) / tw;
      }
      return n;
    };
    if (tiles_at(tw_fb) * K < 2LL * M->n_cu) {
      wclass = TW_NARROW;
      tw_fb = block_tile_width(dt, C, K, TW_NARROW, c.train != 0);
      const int tw3 = block_tile_width(dt, C, K, TW_NARROW3, c.train != 0);
      if (tw3 && tiles_at(tw_fb) * K > 2LL * M->n_cu) {
        wclass = TW_NARROW3;
        tw_fb = tw3;
      }
    }
  }
  hipError_t e;

  // tile geometry for every tile width in use
  int n_tiles_in = 0, n_tiles_blk = 0, n_tiles_fb = 0, n_tiles_ds = 0;
  const TileDesc* d_in = nullptr;
  const TileDesc* d_blk = nullptr;
  const TileDesc* d_fb = nullptr;
  const TileDesc* d_ds = nullptr;
  int64_t n_re = 0;
  if (geo.uniform) {
    n_tiles_in = geo.B * ((geo.F + tw_in - 1) / tw_in);
    n_tiles_blk = geo.B * ((geo.F + tw_blk - 1) / tw_blk);
    if (tw_fb) n_tiles_fb = geo.B * ((geo.F + tw_fb - 1) / tw_fb);
    if (ds) n_tiles_ds = geo.B * ((geo.F + DS_TW - 1) / DS_TW);
    n_re = (int64_t)geo.B * geo.T * geo.F;
  } else {
    std::vector<TileDesc> h;
    auto build = [&](int tw) {
      const size_t first = h.size();
      int64_t base = 0;
      for (int sl = 0; sl < geo.n_slots; ++sl) {
        const int F = geo.F_host[sl];
        for (int f0 = 0; f0 < F; f0 += tw) h.push_back(TileDesc{base, F, f0});
        base += (int64_t)geo.T * F;
      }
      n_re = base;
      return first;
    };
    const size_t o_blk = build(tw_blk);
    n_tiles_blk = (int)(h.size() - o_blk);
    const size_t o_in = tw_in != tw_blk ? build(tw_in) : o_blk;
    n_tiles_in = (int)(tw_in != tw_blk ? h.size() - o_in : n_tiles_blk);
    size_t o_fb = 0, o_ds = 0;
    if (tw_fb) {
      o_fb = build(tw_fb);
      n_tiles_fb = (int)(h.size() - o_fb);
    }
    if (ds) {
      o_ds = build(DS_TW);
      n_tiles_ds = (int)(h.size() - o_ds);
    }
    if (h.size() > ar.max_tiles) return fail(CONET_ESHAPE, "ragged batch needs %zu tiles, capacity %zu", h.size(), ar.max_tiles);
    if (n_re > ar.max_res) return fail(CONET_ESHAPE, "ragged batch has %lld REs, buffers hold %lld", (long long)n_re, (long long)ar.max_res);
    TileDesc* dt_dev = ar.tiles;
    const TileDesc* src = h.data();
    if (geo.tiles_pin && h.size() <= geo.tiles_pin_cap) {
      std::memcpy(geo.tiles_pin, h.data(), h.size() * sizeof(TileDesc));
      src = geo.tiles_pin;
    }
    e = hipMemcpyAsync(dt_dev, src, h.size() * sizeof(TileDesc), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "tile descriptor upload");
    d_blk = dt_dev + o_blk;
    d_in = dt_dev + o_in;
    d_fb = dt_dev + o_fb;
    d_ds = dt_dev + o_ds;
  }
  if (n_tiles_in == 0 || n_tiles_blk == 0) return CONET_OK;

  auto geom = [&](ConvArgs& a, bool in_layer) {
    const int tw = in_layer ? tw_in : tw_blk;
    a.narrow = narrow ? 1 : 0;
    a.T = geo.T;
    a.F = geo.uniform ? geo.F : 0;
    a.tiles_per_slot = geo.uniform ? (geo.F + tw - 1) / tw : 0;
    a.tiles = in_layer ? d_in : d_blk;
  };
  if (geo.uniform && n_re > ar.max_res) return fail(CONET_ESHAPE, "batch has %lld REs, buffers hold %lld", (long long)n_re, (long long)ar.max_res);
  // residual-stream buffers: ping-pong, or one per level when saving for the backward
  int lvl = 0;  // block being launched
  auto actp = [&](int p, int k) -> void* {
    if (!save) return ar.act[p][k];
    return ar.lvl_act[p == (lvl & 1) ? lvl : lvl + 1][k];
  };
  auto hidp = [&](int k) -> void* { return save ? ar.lvl_hid[lvl][k] : ar.hid[k]; };
  if (save && !ar.levels) return fail(CONET_ESTATE, "no per-level buffers");
  unsigned* amax_dev = ar.amax;
  auto read_amax = [&](int n, std::vector<float>& outv) -> conet_status {
    std::vector<unsigned> hbuf(n);
    hipError_t e2 = hipStreamSynchronize(s);
    if (e2 == hipSuccess) e2 = hipMemcpy(hbuf.data(), amax_dev, n * sizeof(unsigned), hipMemcpyDeviceToHost);
    if (e2 != hipSuccess) return hip_fail(e2, "calibration readback");
    outv.resize(n);
    for (int i = 0; i < n; ++i) { float f; std::memcpy(&f, &hbuf[i], 4); outv[i] = f; }
    return CONET_OK;
  };
  auto to_scale = [](float amax) { return amax > 0.f ? amax / E4M3_MAX : 1.0f; };
  if (calib && !geo.uniform) return fail(CONET_EINVAL, "calibration takes a uniform batch");
  if ((calib || save) && geo.grid_rx) return fail(CONET_EINVAL, "calibration and training forwards take features");

  int stage = 0;
  auto mark = [&]() -> hipError_t {
    const int i = stage++;
    return events ? hipEventRecord(events[i], s) : hipSuccess;
  };
  auto add_units = [&](int n) { if (units && stage > 0) units[stage - 1] += n; };

  // ---- input layer
  if (calib) {
    e = hipMemsetAsync(amax_dev, 0, 64 * sizeof(unsigned), s);
    if (e == hipSuccess) e = launch_amax(x, 4, n_re, Ci, nullptr, nullptr, 0, amax_dev, s);
    if (e != hipSuccess) return hip_fail(e, "calibration amax");
    std::vector<float> am;
    conet_status st = read_amax(1, am);
    if (st != CONET_OK) return st;
    sc[0] = to_scale(am[0]);
    calib->push_back(am[0]);
  }
  {
    ConvArgs a = {};
    geom(a, true);
    for (int k = 0; k < K; ++k) {
      a.in[k] = x;
      a.out[k] = actp(0, k);
      a.wpack[k] = ws + lay.w_in[k];
      a.bias[k] = vec + lay.v_bin[k];
      a.wscale[k] = vec + lay.v_wsin[k];
      a.in_qscale[k] = 1.0f / sc[0];
      a.deq[k] = sc[0];
    }
    a.grid_rx = geo.grid_rx;  // features formed while staging the received grid
    e = mark();
    a.inner_branches = K;  // the features are staged once per tile for all branches
    if (e == hipSuccess) e = launch_conv(dt, 0, Ci, C, a, n_tiles_in, 1, s);
    if (e != hipSuccess) return hip_fail(e, "input layer launch");
    add_units(K);
  }

  // the fusion epilogue pass that follows a level's block launches when no block kernel folds
  // the fusion in (by concatenation, or after separable blocks), or that runs the head after
  // an unfused last separable block: reads the stored outputs at out_p, writes A in place
  auto epilogue = [&](int l, bool fuse, bool last, int out_p, const void* main, bool main_f32,
                      const float* scale = nullptr, const float* shift = nullptr) -> conet_status {
    FuseArgs f = {};
    f.main = main;
    f.main_f32 = main_f32 ? 1 : 0;
    for (int k = 1; k < K; ++k) f.sup[k] = actp(out_p, k);
    f.K = K;
    f.wcat = ws + lay.w_cat[l];
    f.bcat = vec + lay.v_bcat[l];
    f.gamma = scale ? scale : vec + lay.v_gamma[l];
    f.beta = shift ? shift : vec + lay.v_beta[l];
    f.norm_affine = c.norm == CONET_NORM_BN;
    f.eps = c.ln_eps;
    f.out = last ? nullptr : actp(out_p, 0);
    f.feedback = fuse && c.feedback && !last;
    f.Wh = vec + lay.v_wh;
    f.bh = vec + lay.v_bh;
    f.llr = last ? llr : nullptr;
    f.m = c.bits_per_symbol;
    f.n_re = n_re;
    const int mode = !fuse ? EPI_NONE : concat ? EPI_CONCAT : c.fusion_op == CONET_FUSE_SUM ? EPI_SUM : EPI_PRODUCT;
    const hipError_t e2 = launch_fuse_epilogue(dt, C, mode, f, s);
    return e2 == hipSuccess ? CONET_OK : hip_fail(e2, "fusion epilogue launch");
  };
  // BatchNorm by batch statistics after block l: mean, then variance of the product over the
  // batch (work-group partials summed in a fixed order), the folded per-channel affine, the
  // running statistics (training forwards only), then the epilogue with that affine. Mean and
  // 1/sqrt(var + eps) stay in the workspace for the backward.
  auto bn_epilogue = [&](int l, bool last, int out_p, const void* main) -> conet_status {
    float* bn = reinterpret_cast<float*>(ws + lay.tr_bn) + (size_t)4 * C * l;
    float* part = reinterpret_cast<float*>(ws + lay.tr_bn_part);
    float* master = reinterpret_cast<float*>(ws + lay.tr_master);
    const int G = bn_stats_grid(n_re);
    BnStatsArgs sa = {};
    sa.main = main;
    for (int k = 1; k < K; ++k) sa.sup[k] = actp(out_p, k);
    sa.K = K; sa.C = C; sa.n_re = n_re; sa.part = part; sa.mean = bn;
    BnFinishArgs fa = {};
    fa.part = part; fa.groups = G; fa.C = C; fa.n_re = n_re;
    fa.eps = c.ln_eps; fa.momentum = CONET_BN_MOMENTUM;
    fa.gamma = vec + lay.v_gamma[l];
    fa.beta = vec + lay.v_beta[l];
    fa.mean = bn; fa.rs = bn + C; fa.scale = bn + 2 * C; fa.shift = bn + 3 * C;
    fa.running_mean = save ? master + M->bo.bn_mean[l] : nullptr;
    fa.running_var = save ? master + M->bo.bn_var[l] : nullptr;
    hipError_t e2 = hipSuccess;
    for (int pass = 0; pass < 2 && e2 == hipSuccess; ++pass) {
      sa.pass = pass;
      fa.pass = pass;
      e2 = launch_bn_stats(dt, sa, G, s);
      if (e2 == hipSuccess) e2 = launch_bn_finish(fa, s);
    }
    if (e2 != hipSuccess) return hip_fail(e2, "BatchNorm statistics");
    return epilogue(l, true, last, out_p, main, false, bn + 2 * C, bn + 3 * C);
  };

  int cur = 0;
  bool fused_prev = false;
  FusedScheduler fsched{M, geo, n_tiles_fb, d_fb, tw_fb, wclass, llr, s, units};
  for (int l = 0; l < L; ++l) {
    lvl = l;
    const bool last = (l == L - 1);
    const bool fuse = (c.fuse_mask >> l) & 1u;
    const int Kl = l < Ls ? K : 1;  // branches that have block l
    if (ds) {  // separable blocks: one launch over the branches, then the epilogue pass
      const int in_p = cur, out_p = 1 - cur;
      const bool main_f32 = last || (fuse && !concat);  // the main output is read unrounded
      const int nk = (last && !fuse) ? 1 : Kl;
      DsArgs d = {};
      d.T = geo.T;
      d.F = geo.uniform ? geo.F : 0;
      d.tiles_per_slot = geo.uniform ? (geo.F + DS_TW - 1) / DS_TW : 0;
      d.tiles = geo.uniform ? nullptr : d_ds;
      for (int k = 0; k < nk; ++k) {
        const float* vb = vec + lay.v_blk[k][l];
        const float* dw = vec + lay.v_dw[k][l];
        const bool mrb = (k == 0 && fused_prev);
        d.x[k] = actp(in_p, k);
        d.out[k] = (k == 0 && main_f32) ? ar.hid[0] : actp(out_p, k);
        d.out_f32[k] = (k == 0 && main_f32) ? 1 : 0;
        d.pre_s[k] = mrb ? nullptr : vb;
        d.pre_o[k] = mrb ? nullptr : vb + C;
        d.dw1[k] = dw;
        d.dw2[k] = dw + 9 * C;
        d.pw1[k] = ws + lay.w1[k][l];
        d.pw2[k] = ws + lay.w2[k][l];
        d.b1[k] = vb + 2 * C;
        d.post_s[k] = vb + 3 * C;
        d.post_o[k] = vb + 4 * C;
        d.b2[k] = vb + 5 * C;
      }
      e = mark();  // (a)
      if (e == hipSuccess) e = launch_ds_block(dt, C, d, n_tiles_ds, nk, s);
      if (e != hipSuccess) return hip_fail(e, "separable block launch");
      add_units(2 * nk);
      e = mark();  // (b)
      if (e != hipSuccess) return hip_fail(e, "event record");
      if (fuse || last) {
        conet_status st = epilogue(l, fuse, last, out_p, d.out[0], main_f32);
        if (st != CONET_OK) return st;
      }
      e = mark();  // (c)
      if (e != hipSuccess) return hip_fail(e, "event record");
      cur = 1 - cur;
      fused_prev = fuse;
      continue;
    }
    // fusion by concatenation, or BatchNorm by batch statistics: the block kernels store every
    // branch output (a training forward keeps the main one where the backward reads it), then
    // the epilogue pass fuses
    const bool bn_lvl = bn_batch && fuse;
    const bool fuse_k = fuse && !concat && !bn_lvl;
    const bool last_k = last && !(fuse && (concat || bn_lvl));
    const int nk = (last_k && !fuse_k) ? 1 : Kl;
    auto out_at = [&](int p, int k) -> void* { return (bn_lvl && save && k == 0) ? ar.lvl_o0[l] : actp(p, k); };
    if (tw_fb) {
      const int in_p = cur, out_p = 1 - cur;
      conet_status st = fsched.block(l, fuse_k, fused_prev, last_k, Kl, [&](int k) { return actp(in_p, k); },
                                     [&](int k) { return out_at(out_p, k); },
                                     [&](int k) -> void* { return save ? hidp(k) : nullptr; },
                                     save ? ar.lvl_o0[l] : nullptr, mark);
      if (st == CONET_OK && fuse && concat) st = epilogue(l, true, last, out_p, actp(out_p, 0), false);
      if (st == CONET_OK && bn_lvl) st = bn_epilogue(l, last, out_p, out_at(out_p, 0));
      if (st != CONET_OK) return st;
      cur = 1 - cur;
      fused_prev = fuse;
      continue;
    }
    ConvArgs a1 = {};
    geom(a1, false);
    for (int k = 0; k < nk; ++k) {
      const float* vb = vec + lay.v_blk[k][l];
      const bool mrb = (k == 0 && fused_prev);
      a1.in[k] = actp(cur, k);
      a1.pre_s[k] = mrb ? nullptr : vb + 0 * C;
      a1.pre_o[k] = mrb ? nullptr : vb + 1 * C;
      a1.bias[k] = vb + 2 * C;
      a1.post_s[k] = vb + 3 * C;
      a1.post_o[k] = vb + 4 * C;
      a1.wscale[k] = vb + 6 * C;
      a1.out[k] = hidp(k);
      a1.wpack[k] = ws + lay.w1[k][l];
    }
    if (calib) {
      // operand of conv 1: max |prologue(x)| per branch, then max |h| per branch
      e = hipMemsetAsync(amax_dev, 0, 64 * sizeof(unsigned), s);
      for (int k = 0; k < nk && e == hipSuccess; ++k)
        e = launch_amax(a1.in[k], 2, n_re, C, a1.pre_s[k], a1.pre_o[k], a1.pre_s[k] ? 1 : 2, amax_dev + k, s);
      if (e != hipSuccess) return hip_fail(e, "calibration amax");
      std::vector<float> am;
      conet_status st = read_amax(nk, am);
      if (st != CONET_OK) return st;
      for (int k = 0; k < nk; ++k) { sc[scale_index(K, L, k, l, 0)] = to_scale(am[k]); calib->push_back(am[k]); }
      for (int k = 0; k < nk; ++k) {
        a1.in_qscale[k] = 1.0f / sc[scale_index(K, L, k, l, 0)];
        a1.deq[k] = sc[scale_index(K, L, k, l, 0)];
        a1.out_qscale[k] = 1.0f;
      }
      ConvArgs ac = a1;
      e = hipMemsetAsync(amax_dev, 0, 64 * sizeof(unsigned), s);
      ac.amax = amax_dev;
      if (e == hipSuccess) e = launch_conv(dt, 1, C, C, ac, n_tiles_blk, nk, s);
      if (e != hipSuccess) return hip_fail(e, "calibration conv");
      st = read_amax(nk, am);
      if (st != CONET_OK) return st;
      for (int k = 0; k < nk; ++k) { sc[scale_index(K, L, k, l, 1)] = to_scale(am[k]); calib->push_back(am[k]); }
    }
    for (int k = 0; k < nk; ++k) {
      a1.in_qscale[k] = 1.0f / sc[scale_index(K, L, k, l, 0)];
      a1.deq[k] = sc[scale_index(K, L, k, l, 0)];
      a1.out_qscale[k] = 1.0f / sc[scale_index(K, L, k, l, 1)];
    }
    e = mark();
    if (e == hipSuccess) e = launch_conv(dt, 1, C, C, a1, n_tiles_blk, nk, s);
    if (e != hipSuccess) return hip_fail(e, "block conv 1 launch");
    add_units(nk);

    ConvArgs a2 = {};
    geom(a2, false);
    for (int k = 0; k < nk; ++k) {
      const float* vb = vec + lay.v_blk[k][l];
      a2.in[k] = hidp(k);
      a2.resid[k] = actp(cur, k);
      a2.wpack[k] = ws + lay.w2[k][l];
      a2.bias[k] = vb + 5 * C;
      a2.wscale[k] = vb + 7 * C;
      a2.deq[k] = sc[scale_index(K, L, k, l, 1)];
      a2.in_qscale[k] = 1.0f / sc[scale_index(K, L, k, l, 1)];
    }
    a2.K = K;
    a2.eps = c.ln_eps;
    a2.gamma = vec + lay.v_gamma[l];
    a2.beta = vec + lay.v_beta[l];
    a2.Wh = vec + lay.v_wh;
    a2.bh = vec + lay.v_bh;
    a2.m = c.bits_per_symbol;
    if (fuse_k) {
      // support branches first (their outputs are stored: the next block's inputs and
      // this block's product operands), then the main branch with the fusion epilogue
      if (K > 1) {
        ConvArgs as = a2;
        for (int k = 1; k < K; ++k) as.out[k] = actp(1 - cur, k);
        as.k_off = 1;
        e = mark();
        if (e == hipSuccess) e = launch_conv(dt, 2, C, C, as, n_tiles_blk, K - 1, s);
        if (e != hipSuccess) return hip_fail(e, "support conv 2 launch");
        add_units(K - 1);
      } else {
        e = mark();
      }
      ConvArgs am = a2;
      for (int k = 1; k < K; ++k) am.sup[k] = actp(1 - cur, k);
      am.out[0] = last_k ? nullptr : actp(1 - cur, 0);
      am.llr = (last_k && !calib) ? llr : nullptr;
      am.save_o0 = save ? ar.lvl_o0[l] : nullptr;
      am.k_off = 0;
      am.fusion_sum = c.fusion_op == CONET_FUSE_SUM;
      am.norm_affine = c.norm == CONET_NORM_BN;
      am.feedback = c.feedback && !last_k;
      e = mark();
      if (e == hipSuccess) e = launch_conv(dt, 4, C, C, am, n_tiles_blk, 1, s);
      if (e != hipSuccess) return hip_fail(e, "fused conv 2 launch");
      add_units(1);
    } else {
      for (int k = 0; k < nk; ++k) a2.out[k] = last_k ? nullptr : out_at(1 - cur, k);
      a2.llr = (last_k && !calib) ? llr : nullptr;
      a2.save_o0 = (save && last_k) ? ar.lvl_o0[l] : nullptr;
      e = mark();
      if (e == hipSuccess) e = launch_conv(dt, 2, C, C, a2, n_tiles_blk, nk, s);
      if (e == hipSuccess) add_units(nk);
      if (e == hipSuccess) e = mark();  // no third launch in an unfused block
      if (e != hipSuccess) return hip_fail(e, "block conv 2 launch");
    }
    if (fuse && concat) {
      conet_status st = epilogue(l, true, last, 1 - cur, actp(1 - cur, 0), false);
      if (st != CONET_OK) return st;
    }
    if (bn_lvl) {
      conet_status st = bn_epilogue(l, last, 1 - cur, out_at(1 - cur, 0));
      if (st != CONET_OK) return st;
    }
    cur = 1 - cur;
    fused_prev = fuse;
  }
  e = mark();
  if (e != hipSuccess) return hip_fail(e, "event record");
  return CONET_OK;
}

}  // namespace conet

using namespace conet;

extern "C" conet_status conet_calibrate(conet_model* M, const float* x, int32_t B, int32_t T, int32_t F, void* stream) {
  if (!M || !x) return fail(CONET_EINVAL, "null argument");
  if (M->cfg.dtype != DT_FP8) return fail(CONET_EINVAL, "calibration applies to FP8 models only");
  if (B < 1 || T < 1 || T > TMAX || F < 1) return fail(CONET_ESHAPE, "bad calibration shape");
  if ((int64_t)B * T * F > M->cfg.max_res) return fail(CONET_ESHAPE, "calibration batch exceeds max_res");
  Geometry geo;
  geo.uniform = true; geo.B = B; geo.T = T; geo.F = F;
  std::vector<float> amax;
  conet_status st = run_forward(M, M->arena, x, geo, nullptr, (hipStream_t)stream, &amax);
  if (st != CONET_OK) return st;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "calibration");
  M->scales_set = true;
  return CONET_OK;
}

extern "C" conet_status conet_forward_profiled(conet_model* M, const float* x, int32_t B, int32_t T, int32_t F,
                                               float* llr, float* stage_ms_host, int32_t* stage_units_host,
                                               int32_t n_stages, void* stream) {
  if (!M || !x || !llr || !stage_ms_host) return fail(CONET_EINVAL, "null argument");
  const int ns = 1 + 3 * M->cfg.blocks;
  if (n_stages != ns) return fail(CONET_EINVAL, "expected %d stages, got %d", ns, n_stages);
  if (B < 1 || T < 1 || T > TMAX || F < 1) return fail(CONET_ESHAPE, "bad shape B=%d T=%d F=%d", B, T, F);
  if ((int64_t)B * T * F > M->cfg.max_res) return fail(CONET_ESHAPE, "B*T*F exceeds max_res");
  if (M->cfg.dtype == DT_FP8 && !M->scales_set) return fail(CONET_ESTATE, "FP8 model needs activation scales");
  std::vector<hipEvent_t> ev(ns + 1, nullptr);
  hipError_t e = hipSuccess;
  for (int i = 0; i <= ns && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
  conet_status st = CONET_OK;
  if (e != hipSuccess) st = hip_fail(e, "hipEventCreate");
  if (st == CONET_OK) {
    Geometry geo;
    geo.uniform = true; geo.B = B; geo.T = T; geo.F = F;
    if (stage_units_host)
      for (int i = 0; i < ns; ++i) stage_units_host[i] = 0;
    st = run_forward(M, M->arena, x, geo, llr, (hipStream_t)stream, nullptr, ev.data(), false, stage_units_host);
  }
  if (st == CONET_OK) {
    e = hipEventSynchronize(ev[ns]);
    for (int i = 0; i < ns && e == hipSuccess; ++i) e = hipEventElapsedTime(&stage_ms_host[i], ev[i], ev[i + 1]);
    if (e != hipSuccess) st = hip_fail(e, "stage timing");
  }
  for (auto& x_ : ev) if (x_) (void)hipEventDestroy(x_);
  return st;
}
