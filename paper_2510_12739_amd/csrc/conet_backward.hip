// Training side of the CoNet-Rx library: workspace layout for training, index maps that
// regenerate the kernels' filter packs from the FP32 master copy, the backward launch
// sequence (reverse-mode through head, LayerNorm, product fusion, residual blocks and
// input layers), bitwise BCE, and Adam.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "conet.h"
#include "conet_model.h"
#include "conet_bwd_block.h"

namespace conet {

void blob_offsets(const conet_config& c, BlobOffsets& bo) {
  const int K = c.branches, L = c.blocks;
  const size_t C = c.channels, Ci = c.in_channels, m = c.bits_per_symbol;
  size_t p = 0;
  for (int k = 0; k < K; ++k) {
    bo.w_in[k] = p; p += C * Ci * 9;
    bo.b_in[k] = p; p += C;
    for (int l = 0; l < L; ++l) {
      bo.s0[k][l] = p; p += C;
      bo.o0[k][l] = p; p += C;
      bo.w1[k][l] = p; p += C * C * 9;
      bo.b1[k][l] = p; p += C;
      bo.s1[k][l] = p; p += C;
      bo.o1[k][l] = p; p += C;
      bo.w2[k][l] = p; p += C * C * 9;
      bo.b2[k][l] = p; p += C;
    }
  }
  for (int l = 0; l < L; ++l) { bo.gamma[l] = p; p += C; bo.beta[l] = p; p += C; }
  bo.wh = p; p += m * C;
  bo.bh = p; p += m;
  if (c.norm == CONET_NORM_BN)
    for (int l = 0; l < L; ++l) { bo.bn_mean[l] = p; p += C; bo.bn_var[l] = p; p += C; }
  bo.n = p;
}

static int elem_bytes(int dtype) { return dtype == DT_F32 ? 4 : 2; }

static int64_t conv_rows_cap(const conet_config& c) { return 4 * (c.max_res / (14 * 16) + 4096); }
static constexpr int FUSE_GRID = 1024, BCE_GRID = 1024, MAX_SEGS = 1024;

size_t train_bytes(const conet_config& c, Layout& lay, size_t base) {
  const int K = c.branches, L = c.blocks;
  const size_t C = c.channels, Ci = c.in_channels, n = n_params(c), R = (size_t)c.max_res;
  size_t off = base;
  auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
  lay.tr_master = take(n * 4);
  lay.tr_grad = take(n * 4);
  lay.tr_m = take(n * 4);
  lay.tr_v = take(n * 4);
  lay.tr_zero = take(std::max(C, Ci) * 4);
  lay.tr_wt_begin = off;
  for (int k = 0; k < K; ++k)
    for (int l = 0; l < L; ++l) {
      lay.tr_wt1[k][l] = take(packed_bytes(c.dtype, C, C));
      lay.tr_wt2[k][l] = take(packed_bytes(c.dtype, C, C));
    }
  lay.tr_wt_end = off;
  lay.tr_map_fwd = take(lay.vec / elem_bytes(c.dtype) * 4);
  lay.tr_map_bwd = take((lay.tr_wt_end - lay.tr_wt_begin) / elem_bytes(c.dtype) * 4);
  lay.tr_map_vec = take(lay.n_vec * 4);
  lay.tr_part_conv_rows = (size_t)conv_rows_cap(c);
  lay.tr_part_conv = take((size_t)K * lay.tr_part_conv_rows * 3 * C * 4);
  lay.tr_part_w = take((size_t)K * 256 * C * 9 * std::max(C, Ci) * 4);
  lay.tr_part_b = take((size_t)K * 256 * C * 4);
  lay.tr_part_fuse = take((size_t)FUSE_GRID * (10 * C + 8) * 4);
  lay.tr_part_bce = take((size_t)BCE_GRID * 4);
  lay.tr_loss = take(256);
  lay.tr_segs = take((size_t)MAX_SEGS * sizeof(ReduceSeg));
  lay.tr_red_tmp_floats = (size_t)K * 64 * 1024 + (size_t)K * 2 * C * 9 * std::max(C, Ci) + 65536;
  lay.tr_red_tmp = take(lay.tr_red_tmp_floats * 4);
  lay.tr_bn = take((size_t)4 * L * C * 4);
  lay.tr_bn_part = take((size_t)1024 * C * 4);
  const size_t t_act = align256(R * C * act_bytes_of(c.dtype));
  lay.tr_levels = off;
  lay.tr_levels_bytes = t_act * ((size_t)(L + 1) * K + (size_t)L * K + L + 4 * (size_t)K);
  off = align256(off + lay.tr_levels_bytes);
  return off - base;
}

// Element index maps: packed element e of a filter pack <- blob index (or -1).
static void pack_index(int dtype, int cin, int cout, size_t w_off, bool transposed, int32_t* idx) {
  const int vec = dtype == DT_F32 ? 4 : 8, cpl = 1;
  const int cpt = cin / vec, nch = 9 * cpt, cps = 4 * cpl, ns = (nch + cps - 1) / cps, NOT = cout / 16;
  for (int s = 0; s < ns; ++s)
    for (int ot = 0; ot < NOT; ++ot)
      for (int lane = 0; lane < 64; ++lane) {
        const size_t base = ((((size_t)s * NOT + ot) * cpl) * 64 + lane) * vec;
        const int r = lane & 15, g = lane >> 4;
        const int o = (r >> 2) * (4 * NOT) + 4 * ot + (r & 3);
        const int ch = (s * 4 + g) * cpl;
        for (int e = 0; e < vec; ++e) {
          int32_t v = -1;
          if (ch < nch) {
            const int tap = ch / cpt, i = (ch % cpt) * vec + e;
            // forward: W[o][i][tap]; input-gradient pack: W'[o'=i][i'=o][tap'] = W[i'][o'][8 - tap']
            v = transposed ? (int32_t)(w_off + ((size_t)i * cout + o) * 9 + (8 - tap))
                           : (int32_t)(w_off + ((size_t)o * cin + i) * 9 + tap);
          }
          idx[base + e] = v;
        }
      }
}

conet_status train_init(conet_model* M) {
  const conet_config& c = M->cfg;
  Layout& lay = M->lay;
  const BlobOffsets& bo = M->bo;
  const int K = c.branches, L = c.blocks, C = c.channels, Ci = c.in_channels, m = c.bits_per_symbol;
  const int eb = elem_bytes(c.dtype);
  std::vector<int32_t> mf(lay.vec / eb, -1), mb((lay.tr_wt_end - lay.tr_wt_begin) / eb, -1), mv(lay.n_vec, -1);
  for (int k = 0; k < K; ++k) {
    pack_index(c.dtype, Ci, C, bo.w_in[k], false, mf.data() + lay.w_in[k] / eb);
    for (int l = 0; l < L; ++l) {
      pack_index(c.dtype, C, C, bo.w1[k][l], false, mf.data() + lay.w1[k][l] / eb);
      pack_index(c.dtype, C, C, bo.w2[k][l], false, mf.data() + lay.w2[k][l] / eb);
      pack_index(c.dtype, C, C, bo.w1[k][l], true, mb.data() + (lay.tr_wt1[k][l] - lay.tr_wt_begin) / eb);
      pack_index(c.dtype, C, C, bo.w2[k][l], true, mb.data() + (lay.tr_wt2[k][l] - lay.tr_wt_begin) / eb);
    }
    for (int i = 0; i < C; ++i) {
      mv[lay.v_bin[k] + i] = (int32_t)(bo.b_in[k] + i);
      for (int l = 0; l < L; ++l) {
        const size_t vb = lay.v_blk[k][l];  // s0 o0 b1 s1 o1 b2 ws1 ws2
        mv[vb + 0 * C + i] = (int32_t)(bo.s0[k][l] + i);
        mv[vb + 1 * C + i] = (int32_t)(bo.o0[k][l] + i);
        mv[vb + 2 * C + i] = (int32_t)(bo.b1[k][l] + i);
        mv[vb + 3 * C + i] = (int32_t)(bo.s1[k][l] + i);
        mv[vb + 4 * C + i] = (int32_t)(bo.o1[k][l] + i);
        mv[vb + 5 * C + i] = (int32_t)(bo.b2[k][l] + i);
      }
    }
  }
  for (int l = 0; l < L; ++l)
    for (int i = 0; i < C; ++i) {
      mv[lay.v_gamma[l] + i] = (int32_t)(bo.gamma[l] + i);
      mv[lay.v_beta[l] + i] = (int32_t)(bo.beta[l] + i);
    }
  for (int i = 0; i < m * C; ++i) mv[lay.v_wh + i] = (int32_t)(bo.wh + i);
  for (int i = 0; i < m; ++i) mv[lay.v_bh + i] = (int32_t)(bo.bh + i);

  uint8_t* ws = M->ws;
  const size_t n = bo.n;
  hipError_t e = hipMemcpy(ws + lay.tr_map_fwd, mf.data(), mf.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ws + lay.tr_map_bwd, mb.data(), mb.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ws + lay.tr_map_vec, mv.data(), mv.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ws + lay.tr_master, M->blob.data(), n * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(ws + lay.tr_m, 0, n * 4);
  if (e == hipSuccess) e = hipMemset(ws + lay.tr_v, 0, n * 4);
  if (e == hipSuccess) e = hipMemset(ws + lay.tr_grad, 0, n * 4);
  if (e == hipSuccess) e = hipMemset(ws + lay.tr_zero, 0, std::max(C, Ci) * 4);
  if (e != hipSuccess) return hip_fail(e, "training set-up");
  // input-gradient packs from the master (the forward packs were written by conet_create)
  e = launch_repack(reinterpret_cast<float*>(ws + lay.tr_master), reinterpret_cast<int32_t*>(ws + lay.tr_map_bwd),
                    ws + lay.tr_wt_begin, (int64_t)mb.size(), c.dtype, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "training repack");

  // per-level buffers
  Arena& ar = M->train_arena;
  ar = M->arena;  // descriptors and counters are shared
  ar.levels = true;
  const size_t t_act = align256((size_t)c.max_res * C * act_bytes_of(c.dtype));
  uint8_t* p = ws + lay.tr_levels;
  for (int l = 0; l <= L; ++l)
    for (int k = 0; k < K; ++k) { ar.lvl_act[l][k] = p; p += t_act; }
  for (int l = 0; l < L; ++l)
    for (int k = 0; k < K; ++k) { ar.lvl_hid[l][k] = p; p += t_act; }
  for (int l = 0; l < L; ++l) { ar.lvl_o0[l] = p; p += t_act; }
  for (int k = 0; k < K; ++k) { ar.g_dO[k] = p; p += t_act; }
  for (int k = 0; k < K; ++k) { ar.g_dc1[k] = p; p += t_act; }
  for (int k = 0; k < K; ++k) { ar.g_dx[0][k] = p; p += t_act; }
  for (int k = 0; k < K; ++k) { ar.g_dx[1][k] = p; p += t_act; }
  return CONET_OK;
}

// Regenerate every filter pack and per-channel vector from the FP32 master.
static hipError_t repack_all(conet_model* M, hipStream_t s) {
  const Layout& lay = M->lay;
  uint8_t* ws = M->ws;
  const int eb = elem_bytes(M->cfg.dtype);
  const float* master = reinterpret_cast<float*>(ws + lay.tr_master);
  hipError_t e = launch_repack(master, reinterpret_cast<int32_t*>(ws + lay.tr_map_fwd), ws, (int64_t)(lay.vec / eb),
                               M->cfg.dtype, s);
  if (e == hipSuccess)
    e = launch_repack(master, reinterpret_cast<int32_t*>(ws + lay.tr_map_bwd), ws + lay.tr_wt_begin,
                      (int64_t)((lay.tr_wt_end - lay.tr_wt_begin) / eb), M->cfg.dtype, s);
  if (e == hipSuccess)
    e = launch_gather(master, reinterpret_cast<int32_t*>(ws + lay.tr_map_vec), reinterpret_cast<float*>(ws + lay.vec),
                      (int64_t)lay.n_vec, s);
  return e;
}

// ---------------------------------------------------------------- backward
static conet_status run_backward(conet_model* M, const float* dllr, hipStream_t s) {
  const conet_config& c = M->cfg;
  const Layout& lay = M->lay;
  const BlobOffsets& bo = M->bo;
  const Arena& ar = M->train_arena;
  uint8_t* ws = M->ws;
  const int K = c.branches, L = c.blocks, C = c.channels, Ci = c.in_channels, dt = c.dtype, m = c.bits_per_symbol;
  float* vec = reinterpret_cast<float*>(ws + lay.vec);
  float* grad = reinterpret_cast<float*>(ws + lay.tr_grad);
  const float* zero = reinterpret_cast<const float*>(ws + lay.tr_zero);
  float* part_conv = reinterpret_cast<float*>(ws + lay.tr_part_conv);
  float* part_w = reinterpret_cast<float*>(ws + lay.tr_part_w);
  float* part_b = reinterpret_cast<float*>(ws + lay.tr_part_b);
  float* part_fuse = reinterpret_cast<float*>(ws + lay.tr_part_fuse);
  ReduceSeg* segs_dev = reinterpret_cast<ReduceSeg*>(ws + lay.tr_segs);
  const int B = (int)M->saved_B, T = M->saved_T, F = M->saved_F;
  const int64_t n_re = (int64_t)B * T * F;
  const int tw_blk = conv_tile_width(dt, C, C);
  const int n_tiles_blk = B * ((F + tw_blk - 1) / tw_blk);
  const int wtw = wgrad_tile_width(dt);
  const int n_tiles_wg = B * ((F + wtw - 1) / wtw);
  auto wg_grid = [&](int nk) { return wgrad_grid(n_tiles_wg, nk, M->n_cu); };
  if ((int64_t)n_tiles_blk * CONV_NW > (int64_t)lay.tr_part_conv_rows)
    return fail(CONET_ESHAPE, "batch needs %lld partial rows, capacity %zu", (long long)n_tiles_blk * CONV_NW,
                lay.tr_part_conv_rows);
  const int conv_rows = n_tiles_blk * CONV_NW;
  // both input-gradient convs of a block in one launch where that kernel exists (BF16, 32 or 64
  // channels) and its two sets of partial rows fit the buffer
  const int tw_bb = bwd_block_tile_width(dt, C);
  const int n_tiles_bb = tw_bb ? B * ((F + tw_bb - 1) / tw_bb) : 0;
  const bool fused_bwd = tw_bb > 0 && 2LL * n_tiles_bb * CONV_NW <= (int64_t)lay.tr_part_conv_rows;
  const int bb_rows = n_tiles_bb * CONV_NW;
  const size_t conv_stride = lay.tr_part_conv_rows * 3 * C;     // floats per branch
  const size_t w_stride = (size_t)256 * C * 9 * std::max(C, Ci);
  const size_t b_stride = (size_t)256 * C;

  // every reduction of this backward, uploaded once; each launch consumes a contiguous range
  std::vector<ReduceSeg> segs;
  struct Range { int first, n, max_cols, max_chunks; size_t tmp_used; };
  std::vector<Range> ranges;
  float* red_tmp = reinterpret_cast<float*>(ws + lay.tr_red_tmp);
  bool tmp_overflow = false;
  auto begin_range = [&]() { ranges.push_back({(int)segs.size(), 0, 0, 0, 0}); };
  auto add = [&](const float* src, float* dst, int rows, int cols, int ld, int map, int cin) {
    Range& r = ranges.back();
    const int chunks = (rows + REDUCE_CHUNK - 1) / REDUCE_CHUNK;
    const size_t need = (size_t)chunks * cols;
    if (r.tmp_used + need > lay.tr_red_tmp_floats) tmp_overflow = true;
    segs.push_back({src, dst, rows, cols, ld, map, cin, red_tmp + r.tmp_used});
    r.tmp_used += need;
    r.n++;
    r.max_cols = std::max(r.max_cols, cols);
    r.max_chunks = std::max(r.max_chunks, chunks);
  };

  hipError_t e = hipMemsetAsync(grad, 0, bo.n * 4, s);
  if (e != hipSuccess) return hip_fail(e, "gradient clear");

  // branches whose block outputs reach the loss: the main net always; the supports at
  // block l if block l is fused or their outputs feed a block above where they do
  int nk_of[LMAX];
  {
    bool sup = false;
    for (int l = L - 1; l >= 0; --l) {
      sup = sup || ((c.fuse_mask >> l) & 1u);
      nk_of[l] = sup ? K : 1;
    }
  }
  // plan the reductions first (so their descriptors are uploaded in one copy)
  for (int l = L - 1; l >= 0; --l) {
    const bool fuse = (c.fuse_mask >> l) & 1u, last = l == L - 1;
    const int nk = nk_of[l];
    if (fuse || last) {
      begin_range();
      if (fuse) {
        add(part_fuse + 0, grad + bo.gamma[l], FUSE_GRID, C, 10 * C + 8, 0, 0);
        add(part_fuse + C, grad + bo.beta[l], FUSE_GRID, C, 10 * C + 8, 0, 0);
      }
      if (last) {
        add(part_fuse + 2 * C, grad + bo.wh, FUSE_GRID, m * C, 10 * C + 8, 0, 0);
        add(part_fuse + 10 * C, grad + bo.bh, FUSE_GRID, m, 10 * C + 8, 0, 0);
      }
    }
    if (fused_bwd) {  // one launch: rows [0, bb_rows) hold the s1 / o1 sums, the next bb_rows the s0 / o0 sums
      begin_range();
      for (int k = 0; k < nk; ++k) {
        float* pk = part_conv + k * conv_stride;
        add(pk + 0 * C, grad + bo.s1[k][l], bb_rows, C, 3 * C, 0, 0);
        add(pk + 1 * C, grad + bo.o1[k][l], bb_rows, C, 3 * C, 0, 0);
        add(pk + (size_t)bb_rows * 3 * C + 0 * C, grad + bo.s0[k][l], bb_rows, C, 3 * C, 0, 0);
        add(pk + (size_t)bb_rows * 3 * C + 1 * C, grad + bo.o0[k][l], bb_rows, C, 3 * C, 0, 0);
      }
    } else {
      begin_range();
      for (int k = 0; k < nk; ++k) {
        add(part_conv + k * conv_stride + 0 * C, grad + bo.s1[k][l], conv_rows, C, 3 * C, 0, 0);
        add(part_conv + k * conv_stride + 1 * C, grad + bo.o1[k][l], conv_rows, C, 3 * C, 0, 0);
      }
    }
    begin_range();
    for (int k = 0; k < nk; ++k) {
      add(part_w + k * w_stride, grad + bo.w2[k][l], wg_grid(nk), C * 9 * C, C * 9 * C, 1, C);
      add(part_b + k * b_stride, grad + bo.b2[k][l], wg_grid(nk), C, C, 0, 0);
    }
    if (!fused_bwd) {
      begin_range();
      for (int k = 0; k < nk; ++k) {
        add(part_conv + k * conv_stride + 0 * C, grad + bo.s0[k][l], conv_rows, C, 3 * C, 0, 0);
        add(part_conv + k * conv_stride + 1 * C, grad + bo.o0[k][l], conv_rows, C, 3 * C, 0, 0);
      }
    }
    begin_range();
    for (int k = 0; k < nk; ++k) {
      add(part_w + k * w_stride, grad + bo.w1[k][l], wg_grid(nk), C * 9 * C, C * 9 * C, 1, C);
      add(part_b + k * b_stride, grad + bo.b1[k][l], wg_grid(nk), C, C, 0, 0);
    }
  }
  begin_range();
  for (int k = 0; k < nk_of[0]; ++k) {
    add(part_w + k * w_stride, grad + bo.w_in[k], wg_grid(nk_of[0]), C * 9 * Ci, C * 9 * Ci, 1, Ci);
    add(part_b + k * b_stride, grad + bo.b_in[k], wg_grid(nk_of[0]), C, C, 0, 0);
  }
  if ((int)segs.size() > MAX_SEGS) return fail(CONET_EINVAL, "too many reductions");
  if (tmp_overflow) return fail(CONET_ESHAPE, "reduction scratch too small for this batch");
  e = hipMemcpyAsync(segs_dev, segs.data(), segs.size() * sizeof(ReduceSeg), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "reduction descriptors");

  auto reduce = [&](size_t ri) -> hipError_t {
    const Range& r = ranges[ri];
    return launch_reduce(segs_dev + r.first, r.n, r.max_cols, r.max_chunks, s);
  };

  // gradient w.r.t. the input of block l+1 (level l+1), per branch; null above the last block
  const void* dx_next[KMAX_ARGS] = {};
  int dxbuf = 0;
  size_t ri = 0;
  for (int l = L - 1; l >= 0; --l) {
    const bool fuse = (c.fuse_mask >> l) & 1u, last = l == L - 1;
    const bool fused_prev = l > 0 && ((c.fuse_mask >> (l - 1)) & 1u);
    const int nk = nk_of[l];
    // gradients of the block outputs O[k]
    const void* dO[KMAX_ARGS] = {};
    if (fuse || last) {
      FuseBwdArgs fa = {};
      fa.dllr = last ? dllr : nullptr;
      fa.dA = last ? nullptr : dx_next[0];
      for (int k = 0; k < K; ++k) {
        fa.O[k] = k == 0 ? ar.lvl_o0[l] : ar.lvl_act[l + 1][k];
        fa.dnext[k] = (!last && k > 0) ? dx_next[k] : nullptr;
        fa.dO[k] = (k < nk) ? ar.g_dO[k] : nullptr;
      }
      if (!fuse) fa.O[0] = ar.lvl_o0[l];  // unfused last block: the head reads O[0] itself
      fa.gamma = vec + lay.v_gamma[l];
      fa.beta = vec + lay.v_beta[l];
      fa.Wh = vec + lay.v_wh;
      fa.m = m; fa.K = fuse ? K : 1; fa.C = C; fa.fused = fuse; fa.head = last;
      fa.eps = c.ln_eps;
      fa.n_re = n_re;
      fa.part = part_fuse;
      fa.a_out = last ? ar.g_dc1[0] : nullptr;  // the head's input (g_dc1 is free until conv 2's adjoint)
      HeadWgradArgs hw = {};
      hw.A = ar.g_dc1[0]; hw.dllr = dllr; hw.m = m; hw.n_re = n_re;
      hw.part = part_fuse; hw.ld = 10 * C + 8; hw.col0 = 2 * C;
      auto head_wgrad = [&]() { return last ? launch_head_wgrad(dt, C, hw, FUSE_GRID, s) : hipSuccess; };
      if (fuse && c.norm == CONET_NORM_BN) {  // batch statistics: two passes around the reduction
        const float* bn = reinterpret_cast<const float*>(ws + lay.tr_bn) + (size_t)4 * C * l;
        fa.bn_mu = bn;
        fa.bn_rs = bn + C;
        fa.bn_pass = 1;
        e = launch_fuse_bwd(dt, fa, FUSE_GRID, s);
        if (e == hipSuccess) e = head_wgrad();
        if (e == hipSuccess) e = reduce(ri);
        fa.bn_pass = 2;
        fa.bn_dgamma = grad + bo.gamma[l];
        fa.bn_dbeta = grad + bo.beta[l];
        fa.part = nullptr;
        fa.a_out = nullptr;
        if (e == hipSuccess) e = launch_fuse_bwd(dt, fa, FUSE_GRID, s);
      } else {
        e = launch_fuse_bwd(dt, fa, FUSE_GRID, s);
        if (e == hipSuccess) e = head_wgrad();
        if (e == hipSuccess) e = reduce(ri);
      }
      if (e != hipSuccess) return hip_fail(e, "head / fusion backward");
      for (int k = 0; k < nk; ++k) dO[k] = ar.g_dO[k];
    } else {
      for (int k = 0; k < K; ++k) dO[k] = dx_next[k];
    }
    if (fuse || last) ++ri;
    // W2, b2 (independent of the input gradients)
    WgradArgs w2 = {};
    for (int k = 0; k < nk; ++k) {
      w2.dout[k] = dO[k];
      w2.in[k] = ar.lvl_hid[l][k];
      w2.part_w[k] = part_w + k * w_stride;
      w2.part_b[k] = part_b + k * b_stride;
    }
    w2.prologue = 0;
    w2.T = T; w2.F = F; w2.tiles_per_slot = (F + wtw - 1) / wtw; w2.n_tiles = n_tiles_wg; w2.grid = wg_grid(nk);
    if (fused_bwd) {  // through both convs: dc1 and dx of the block input
      BwdBlockArgs bb = {};
      bb.T = T; bb.F = F; bb.tiles_per_slot = (F + tw_bb - 1) / tw_bb;
      bb.rows = bb_rows;
      bb.mask_out = l == 0;
      for (int k = 0; k < nk; ++k) {
        const float* vb = vec + lay.v_blk[k][l];
        const bool mrb = (k == 0 && fused_prev);
        bb.dO[k] = dO[k];
        bb.h[k] = ar.lvl_hid[l][k];
        bb.x[k] = ar.lvl_act[l][k];
        bb.wt1[k] = ws + lay.tr_wt1[k][l];
        bb.wt2[k] = ws + lay.tr_wt2[k][l];
        bb.s1[k] = vb + 3 * C;
        bb.o1[k] = vb + 4 * C;
        bb.s0[k] = mrb ? nullptr : vb + 0 * C;
        bb.o0[k] = mrb ? nullptr : vb + 1 * C;
        bb.dc1[k] = ar.g_dc1[k];
        bb.dx[k] = ar.g_dx[dxbuf][k];
        bb.part[k] = part_conv + k * conv_stride;
      }
      e = launch_bwd_block(dt, C, bb, n_tiles_bb, nk, s);
      if (e == hipSuccess) e = reduce(ri++);
      if (e != hipSuccess) return hip_fail(e, "block input gradient");
      e = launch_wgrad(dt, false, C, C, w2, nk, s);
      if (e == hipSuccess) e = reduce(ri++);
      if (e != hipSuccess) return hip_fail(e, "conv 2 filter gradient");
    } else {
      // through the second conv: dc1
      ConvArgs a5 = {};
      a5.T = T; a5.F = F; a5.tiles_per_slot = (F + tw_blk - 1) / tw_blk;
      for (int k = 0; k < nk; ++k) {
        const float* vb = vec + lay.v_blk[k][l];
        a5.in[k] = dO[k];
        a5.wpack[k] = ws + lay.tr_wt2[k][l];
        a5.bias[k] = zero;
        a5.wscale[k] = zero;
        a5.aux[k] = ar.lvl_hid[l][k];
        a5.post_s[k] = vb + 3 * C;
        a5.post_o[k] = vb + 4 * C;
        a5.out[k] = ar.g_dc1[k];
        a5.part[k] = part_conv + k * conv_stride;
      }
      e = launch_conv(dt, 5, C, C, a5, n_tiles_blk, nk, s);
      if (e == hipSuccess) e = reduce(ri++);
      if (e != hipSuccess) return hip_fail(e, "conv 2 input gradient");
      e = launch_wgrad(dt, false, C, C, w2, nk, s);
      if (e == hipSuccess) e = reduce(ri++);
      if (e != hipSuccess) return hip_fail(e, "conv 2 filter gradient");
      // through the first conv: dx of the block input
      ConvArgs a6 = {};
      a6.T = T; a6.F = F; a6.tiles_per_slot = (F + tw_blk - 1) / tw_blk;
      for (int k = 0; k < nk; ++k) {
        const float* vb = vec + lay.v_blk[k][l];
        const bool mrb = (k == 0 && fused_prev);
        a6.in[k] = ar.g_dc1[k];
        a6.wpack[k] = ws + lay.tr_wt1[k][l];
        a6.bias[k] = zero;
        a6.wscale[k] = zero;
        a6.aux[k] = ar.lvl_act[l][k];
        a6.pre_s[k] = mrb ? nullptr : vb + 0 * C;
        a6.pre_o[k] = mrb ? nullptr : vb + 1 * C;
        a6.resid[k] = dO[k];
        a6.out[k] = ar.g_dx[dxbuf][k];
        a6.part[k] = part_conv + k * conv_stride;
      }
      a6.mask_out = l == 0;
      e = launch_conv(dt, 6, C, C, a6, n_tiles_blk, nk, s);
      if (e == hipSuccess) e = reduce(ri++);
      if (e != hipSuccess) return hip_fail(e, "conv 1 input gradient");
    }
    // W1, b1 (In = the block's pre-activation, recomputed while staging)
    WgradArgs w1 = {};
    for (int k = 0; k < nk; ++k) {
      const float* vb = vec + lay.v_blk[k][l];
      const bool mrb = (k == 0 && fused_prev);
      w1.dout[k] = ar.g_dc1[k];
      w1.in[k] = ar.lvl_act[l][k];
      w1.pre_s[k] = mrb ? nullptr : vb + 0 * C;
      w1.pre_o[k] = mrb ? nullptr : vb + 1 * C;
      w1.part_w[k] = part_w + k * w_stride;
      w1.part_b[k] = part_b + k * b_stride;
    }
    w1.prologue = 1;
    w1.T = T; w1.F = F; w1.tiles_per_slot = (F + wtw - 1) / wtw; w1.n_tiles = n_tiles_wg; w1.grid = wg_grid(nk);
    e = launch_wgrad(dt, false, C, C, w1, nk, s);
    if (e == hipSuccess) e = reduce(ri++);
    if (e != hipSuccess) return hip_fail(e, "conv 1 filter gradient");
    for (int k = 0; k < K; ++k) dx_next[k] = k < nk ? ar.g_dx[dxbuf][k] : nullptr;
    dxbuf ^= 1;
  }
  // input layers: dz = dx_0 * [a0 > 0] (applied by the last input-gradient conv)
  WgradArgs wi = {};
  for (int k = 0; k < K; ++k) {
    wi.dout[k] = dx_next[k];
    wi.in[k] = M->saved_x;
    wi.part_w[k] = part_w + k * w_stride;
    wi.part_b[k] = part_b + k * b_stride;
  }
  wi.prologue = 0;
  wi.T = T; wi.F = F; wi.tiles_per_slot = (F + wtw - 1) / wtw; wi.n_tiles = n_tiles_wg; wi.grid = wg_grid(nk_of[0]);
  e = launch_wgrad(dt, true, Ci, C, wi, nk_of[0], s);
  if (e == hipSuccess) e = reduce(ri++);
  if (e != hipSuccess) return hip_fail(e, "input layer filter gradient");
  return CONET_OK;
}

}  // namespace conet

using namespace conet;

extern "C" {

conet_status conet_backward(conet_model* M, const float* dllr, void* stream) {
  if (!M || !dllr) return fail(CONET_EINVAL, "null argument");
  if (!M->cfg.train) return fail(CONET_ESTATE, "model was not created with train = 1");
  if (!M->saved) return fail(CONET_ESTATE, "backward needs a forward with save_for_backward = 1 first");
  return run_backward(M, dllr, (hipStream_t)stream);
}

conet_status conet_grads(conet_model* M, float** grads_dev, size_t* n) {
  if (!M || !grads_dev || !n) return fail(CONET_EINVAL, "null argument");
  if (!M->cfg.train) return fail(CONET_ESTATE, "model was not created with train = 1");
  *grads_dev = reinterpret_cast<float*>(M->ws + M->lay.tr_grad);
  *n = M->bo.n;
  return CONET_OK;
}

conet_status conet_master_weights(conet_model* M, float** weights_dev, size_t* n) {
  if (!M || !weights_dev || !n) return fail(CONET_EINVAL, "null argument");
  if (!M->cfg.train) return fail(CONET_ESTATE, "model was not created with train = 1");
  *weights_dev = reinterpret_cast<float*>(M->ws + M->lay.tr_master);
  *n = M->bo.n;
  return CONET_OK;
}

conet_status conet_adam_step(conet_model* M, float lr, float b1, float b2, float eps, void* stream) {
  if (!M) return fail(CONET_EINVAL, "null model");
  if (!M->cfg.train) return fail(CONET_ESTATE, "model was not created with train = 1");
  if (!(lr >= 0.f) || !(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
    return fail(CONET_EINVAL, "bad Adam hyper-parameters");
  const Layout& lay = M->lay;
  uint8_t* ws = M->ws;
  const int t = ++M->adam_steps;
  const float bc1 = 1.f - std::pow(b1, (float)t), bc2 = 1.f - std::pow(b2, (float)t);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_adam(reinterpret_cast<float*>(ws + lay.tr_master), reinterpret_cast<float*>(ws + lay.tr_grad),
                             reinterpret_cast<float*>(ws + lay.tr_m), reinterpret_cast<float*>(ws + lay.tr_v),
                             (int64_t)M->bo.n, lr, b1, b2, eps, bc1, bc2, s);
  if (e == hipSuccess) e = repack_all(M, s);
  if (e != hipSuccess) return hip_fail(e, "Adam step");
  M->saved = false;  // the saved activations belong to the old weights
  return CONET_OK;
}

conet_status conet_get_weights(conet_model* M, float* w, size_t n) {
  if (!M || !w) return fail(CONET_EINVAL, "null argument");
  if (n != M->bo.n) return fail(CONET_EINVAL, "expected %zu weights, got %zu", M->bo.n, n);
  if (!M->cfg.train) {
    std::copy(M->blob.begin(), M->blob.end(), w);
    return CONET_OK;
  }
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(w, M->ws + M->lay.tr_master, n * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "weight readback");
  return CONET_OK;
}

conet_status conet_save_train_state(conet_model* M, float* master, float* m, float* v, size_t n, int32_t* steps) {
  if (!M || !master || !m || !v || !steps) return fail(CONET_EINVAL, "null argument");
  if (!M->cfg.train) return fail(CONET_ESTATE, "model was not created with train = 1");
  if (n != M->bo.n) return fail(CONET_EINVAL, "expected %zu values per tensor, got %zu", M->bo.n, n);
  const Layout& lay = M->lay;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(master, M->ws + lay.tr_master, n * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(m, M->ws + lay.tr_m, n * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(v, M->ws + lay.tr_v, n * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "training state readback");
  *steps = M->adam_steps;
  return CONET_OK;
}

conet_status conet_load_train_state(conet_model* M, const float* master, const float* m, const float* v, size_t n,
                                    int32_t steps) {
  if (!M || !master || !m || !v) return fail(CONET_EINVAL, "null argument");
  if (!M->cfg.train) return fail(CONET_ESTATE, "model was not created with train = 1");
  if (n != M->bo.n) return fail(CONET_EINVAL, "expected %zu values per tensor, got %zu", M->bo.n, n);
  if (steps < 0) return fail(CONET_EINVAL, "negative Adam step count");
  const Layout& lay = M->lay;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(M->ws + lay.tr_master, master, n * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M->ws + lay.tr_m, m, n * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(M->ws + lay.tr_v, v, n * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = repack_all(M, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "training state upload");
  M->adam_steps = steps;
  M->saved = false;
  return CONET_OK;
}

conet_status conet_bce(conet_model* M, const float* llr, const uint8_t* bits, const uint8_t* data_mask, int32_t B,
                       int32_t T, int32_t F, int64_t n_data_per_slot, float* dllr, float* loss_dev, void* stream) {
  if (!M || !llr || !bits || !data_mask || !dllr || !loss_dev) return fail(CONET_EINVAL, "null argument");
  if (!M->cfg.train) return fail(CONET_ESTATE, "model was not created with train = 1");
  if (B < 1 || T < 1 || T > TMAX || F < 1) return fail(CONET_ESHAPE, "bad shape");
  if (n_data_per_slot < 1 || n_data_per_slot > (int64_t)T * F) return fail(CONET_EINVAL, "bad data RE count");
  const int m = M->cfg.bits_per_symbol;
  float* part = reinterpret_cast<float*>(M->ws + M->lay.tr_part_bce);
  const float inv = (float)(1.0 / ((double)B * (double)n_data_per_slot * (double)m));
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_bce(llr, bits, data_mask, (int64_t)B * T * F, T, F, m, inv, dllr, part, BCE_GRID, s);
  if (e == hipSuccess) e = launch_sum(part, BCE_GRID, loss_dev, s);
  if (e != hipSuccess) return hip_fail(e, "BCE");
  return CONET_OK;
}

}  // extern "C"
