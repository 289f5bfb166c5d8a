// C-ABI host side of the CoNet-Rx library: configuration checks, filter packing into
// the MFMA fragment order, workspace layout, and the launch sequence of a forward pass.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "conet.h"
#include "conet_common.h"
#include "conet_kernels.h"
#include "conet_model.h"

namespace conet {

thread_local std::string g_last_error;

conet_status fail(conet_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

conet_status hip_fail(hipError_t e, const char* what) {
  return fail(CONET_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ---------------------------------------------------------------- host rounding
uint16_t bf16_bits(float v) {
  uint32_t u;
  memcpy(&u, &v, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Saturating round-to-nearest-even onto OCP e4m3fn (bias 7, 3 mantissa bits, max 448).
uint8_t e4m3_bits(float v) {
  const uint8_t sign = std::signbit(v) ? 0x80 : 0x00;
  double a = std::fabs((double)v);
  if (!(a == a)) return 0x7f;
  if (a > 448.0) a = 448.0;
  if (a == 0.0) return sign;
  int e = (int)std::floor(std::log2(a));
  if (e < -6) e = -6;
  const double q = std::ldexp(1.0, e - 3);
  double n = std::nearbyint(a / q);  // default rounding mode: ties to even
  if (n >= 16.0) { n = 8.0; ++e; }   // rounded up into the next binade
  if (e == -6 && n < 8.0) return (uint8_t)(sign | (uint8_t)n);  // subnormal: mantissa = n
  const int be = e + 7;
  return (uint8_t)(sign | (be << 3) | ((int)n - 8));
}

// ---------------------------------------------------------------- fragment packing
struct OpFmt { int vec, cpl, esize; };
static OpFmt op_fmt(int dtype) {
  switch (dtype) {
    case DT_F32: return {4, 1, 4};
    case DT_BF16: return {8, 1, 2};
    default: return {16, 2, 1};  // DT_FP8
  }
}

size_t packed_bytes(int dtype, int cin, int cout) {
  const OpFmt f = op_fmt(dtype);
  const int cpt = cin / f.vec, nch = 9 * cpt, cps = 4 * f.cpl;
  const int ns = (nch + cps - 1) / cps;
  return (size_t)ns * (cout / 16) * f.cpl * 64 * 16;
}

// W: [cout][cin][3][3] FP32. Lane l of o-tile ot supplies filter row
// o = (r/4)*(4*NOT) + 4*ot + r%4 (r = l%16) for chunk (s*4 + l/16)*CPL + c.
void pack_filter(int dtype, int cin, int cout, const float* W, uint8_t* dst, float* wscale) {
  const OpFmt f = op_fmt(dtype);
  const int cpt = cin / f.vec, nch = 9 * cpt, cps = 4 * f.cpl, ns = (nch + cps - 1) / cps;
  const int NOT = cout / 16;
  std::vector<float> sc(cout, 1.0f);
  if (dtype == DT_FP8) {
    for (int o = 0; o < cout; ++o) {
      float amax = 0.f;
      for (int i = 0; i < cin * 9; ++i) amax = std::max(amax, std::fabs(W[(size_t)o * cin * 9 + i]));
      sc[o] = amax > 0.f ? amax / 448.0f : 1.0f;
    }
  }
  if (wscale) for (int o = 0; o < cout; ++o) wscale[o] = sc[o];
  for (int s = 0; s < ns; ++s)
    for (int ot = 0; ot < NOT; ++ot)
      for (int c = 0; c < f.cpl; ++c)
        for (int lane = 0; lane < 64; ++lane) {
          uint8_t* out = dst + ((((size_t)s * NOT + ot) * f.cpl + c) * 64 + lane) * 16;
          memset(out, 0, 16);
          const int r = lane & 15, g = lane >> 4;
          const int o = (r >> 2) * (4 * NOT) + 4 * ot + (r & 3);
          const int ch = (s * 4 + g) * f.cpl + c;
          if (ch >= nch) continue;
          const int tap = ch / cpt, c0 = (ch % cpt) * f.vec;
          for (int e = 0; e < f.vec; ++e) {
            const float w = W[(((size_t)o * cin + c0 + e) * 3 + tap / 3) * 3 + tap % 3];
            switch (dtype) {
              case DT_F32: memcpy(out + 4 * e, &w, 4); break;
              case DT_BF16: { uint16_t b = bf16_bits(w); memcpy(out + 2 * e, &b, 2); } break;
              default: out[e] = e4m3_bits(w / sc[o]); break;  // DT_FP8
            }
          }
        }
}

// Fragments of the 32x32 MFMAs: [s][ot][lane][CPL x 16 B] for K step s and output tile ot
// (32 filter rows), with CPL = 2 chunks of 16 channels per lane per step (FP8, 32x32x64) or
// 1 chunk of 8 channels (BF16, 32x32x16). Lane half h = l/32 walks the hc = cin/2 / (channels
// per chunk) chunks of channels h*cin/2 .. (h+1)*cin/2 - 1 of every tap in the sequence
// u = 0 .. 9 hc - 1 (tap u / hc, chunk hc h + u % hc); lane l supplies row r = l%32 with the
// chunks u = CPL s .. CPL s + CPL - 1 (past the end: zero). Row r of tile ot is filter
// o = ((r/4)%2) (cout/2) + 16 ot + 4 (r/8) + r%4, so that the accumulator rows a lane holds
// (8j + 4(l/32) + q) are the cout/2 contiguous channels from (l/32) (cout/2).
// wscale: the per-output-channel scales pack_filter chose (FP8; unused for BF16).
struct Frag32 { int cpl, chc, esize; };
static Frag32 frag32(int dtype) { return dtype == DT_FP8 ? Frag32{2, 16, 1} : Frag32{1, 8, 2}; }

size_t packed_bytes32(int dtype, int cin, int cout) {
  const Frag32 f = frag32(dtype);
  const int nu = 9 * (cin / 2 / f.chc), ns = (nu + f.cpl - 1) / f.cpl;
  return (size_t)ns * (cout / 32) * 64 * 16 * f.cpl;
}

void pack_filter32(int dtype, int cin, int cout, const float* W, const float* wscale, uint8_t* dst) {
  const Frag32 f = frag32(dtype);
  const int hc = cin / 2 / f.chc, nu = 9 * hc, ns = (nu + f.cpl - 1) / f.cpl, NOT = cout / 32;
  const int lane_bytes = 16 * f.cpl;
  for (int s = 0; s < ns; ++s)
    for (int ot = 0; ot < NOT; ++ot)
      for (int lane = 0; lane < 64; ++lane) {
        uint8_t* out = dst + (((size_t)s * NOT + ot) * 64 + lane) * lane_bytes;
        memset(out, 0, lane_bytes);
        const int r = lane & 31, h = lane >> 5;
        const int o = ((r >> 2) & 1) * (cout / 2) + 16 * ot + 4 * (r >> 3) + (r & 3);
        for (int cc = 0; cc < f.cpl; ++cc) {
          const int u = f.cpl * s + cc;
          if (u >= nu) continue;  // padding taps: weight 0
          const int tap = u / hc, c0 = (hc * h + u % hc) * f.chc;
          for (int e = 0; e < f.chc; ++e) {
            const float w = W[(((size_t)o * cin + c0 + e) * 3 + tap / 3) * 3 + tap % 3];
            if (dtype == DT_FP8) {
              out[16 * cc + e] = e4m3_bits(w / wscale[o]);
            } else {
              const uint16_t bb = bf16_bits(w);
              memcpy(out + 16 * cc + 2 * e, &bb, 2);
            }
          }
        }
      }
}

// ---------------------------------------------------------------- layout
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static int act_bytes(int dtype) { return dtype == DT_F32 ? 4 : 2; }
size_t act_bytes_of(int dtype) { return (size_t)act_bytes(dtype); }
// middle-activation buffers: the two-conv path's h; separable blocks keep h on chip and use
// branch 0's buffer for the FP32 main output a fusion or the head reads
static int hid_bytes(const conet_config& c) {
  if (c.block_type == CONET_BLOCK_SEPARABLE) return 4;
  return c.dtype == DT_F32 ? 4 : (c.dtype == DT_BF16 ? 2 : 1);
}

static size_t block_params(const conet_config& c) {
  const size_t C = c.channels;
  return c.block_type == CONET_BLOCK_SEPARABLE ? 6 * C + 2 * (9 * C + C * C) : 6 * C + 2 * 9 * C * C;
}

size_t n_params(const conet_config& c) {
  const size_t K = c.branches, L = c.blocks, C = c.channels, Ci = c.in_channels, m = c.bits_per_symbol;
  const size_t bn = c.norm == CONET_NORM_BN ? 2 * L * C : 0;  // running mean and variance per block
  const size_t cat = c.fusion_op == CONET_FUSE_CONCAT ? L * (C * K * C + C) : 0;
  const size_t blocks = L + (K - 1) * (size_t)support_depth(c);
  return K * (C * Ci * 9 + C) + blocks * block_params(c) + 2 * L * C + m * C + m + cat + bn;
}

conet_status check_config(const conet_config* c) {
  if (!c) return fail(CONET_EINVAL, "null config");
  if (c->branches < 1 || c->branches > KMAX_ARGS) return fail(CONET_EINVAL, "branches must be 1..8 (got %d)", c->branches);
  if (c->blocks < 1 || c->blocks > 32) return fail(CONET_EINVAL, "blocks must be 1..32 (got %d)", c->blocks);
  if (c->bits_per_symbol < 1 || c->bits_per_symbol > 8) return fail(CONET_EINVAL, "bits_per_symbol must be 1..8");
  if (c->dtype != DT_F32 && c->dtype != DT_BF16 && c->dtype != DT_FP8) return fail(CONET_EINVAL, "unsupported dtype %d", c->dtype);
  if (!conv_supported(c->dtype, c->in_channels, c->channels))
    return fail(CONET_EINVAL, "no kernel for C_in=%d -> C=%d at dtype %d", c->in_channels, c->channels, c->dtype);
  if (!conv_supported(c->dtype, c->channels, c->channels))
    return fail(CONET_EINVAL, "no kernel for C=%d -> C=%d at dtype %d", c->channels, c->channels, c->dtype);
  if (c->train != 0 && c->train != 1) return fail(CONET_EINVAL, "train must be 0 or 1");
  if (c->fusion_op != CONET_FUSE_PRODUCT && c->fusion_op != CONET_FUSE_SUM && c->fusion_op != CONET_FUSE_CONCAT)
    return fail(CONET_EINVAL, "fusion_op must be CONET_FUSE_PRODUCT, CONET_FUSE_SUM or CONET_FUSE_CONCAT");
  if (c->support_blocks < 0 || c->support_blocks > c->blocks)
    return fail(CONET_EINVAL, "support_blocks must be 0..L (got %d)", c->support_blocks);
  if (c->block_type != CONET_BLOCK_STANDARD && c->block_type != CONET_BLOCK_SEPARABLE)
    return fail(CONET_EINVAL, "block_type must be CONET_BLOCK_STANDARD or CONET_BLOCK_SEPARABLE");
  if (c->block_type == CONET_BLOCK_SEPARABLE && !ds_supported(c->dtype, c->channels))
    return fail(CONET_EINVAL, "separable blocks run in FP32 or BF16 with C = 32 or 64");
  if (c->fusion_op == CONET_FUSE_CONCAT && !concat_supported(c->dtype, c->channels, c->branches))
    return fail(CONET_EINVAL, "fusion by concatenation runs in FP32 or BF16 with C = 32 or 64 and K <= 4");
  if (c->feedback != 0 && c->feedback != 1) return fail(CONET_EINVAL, "feedback must be 0 or 1");
  if (c->norm != CONET_NORM_LN && c->norm != CONET_NORM_BN) return fail(CONET_EINVAL, "norm must be CONET_NORM_LN or CONET_NORM_BN");
  if (c->train) {
    if (c->dtype != DT_F32 && c->dtype != DT_BF16) return fail(CONET_EINVAL, "training runs in FP32 or BF16");
    if (c->channels != 16 && c->channels != 32 && c->channels != 64)
      return fail(CONET_EINVAL, "training supports C = 16, 32, 64");
    if (c->in_channels != 16 && c->in_channels != 32) return fail(CONET_EINVAL, "training supports C_in = 16, 32");
    if (c->branches > 4) return fail(CONET_EINVAL, "training supports K <= 4");
    if (c->blocks > 16) return fail(CONET_EINVAL, "training supports L <= 16");
    if (c->fusion_op != CONET_FUSE_PRODUCT || c->feedback)
      return fail(CONET_EINVAL, "training supports product fusion without feedback");
    if (c->norm == CONET_NORM_BN && c->channels != 32 && c->channels != 64)
      return fail(CONET_EINVAL, "training with BatchNorm supports C = 32, 64");
    if (support_depth(*c) != c->blocks || c->block_type != CONET_BLOCK_STANDARD)
      return fail(CONET_EINVAL, "training supports standard blocks and support branches of depth L");
  }
  if (c->max_res < 1) return fail(CONET_EINVAL, "max_res must be positive");
  if (!(c->ln_eps > 0.f)) return fail(CONET_EINVAL, "ln_eps must be positive");
  if (c->blocks < 32 && (c->fuse_mask >> c->blocks) != 0) return fail(CONET_EINVAL, "fuse_mask has bits beyond L");
  if (support_depth(*c) < 32 && (c->fuse_mask >> support_depth(*c)) != 0)
    return fail(CONET_EINVAL, "fuse_mask has bits beyond the support branches' %d blocks", support_depth(*c));
  return CONET_OK;
}

size_t arena_bytes(const conet_config& c, int64_t max_res) {
  const size_t R = (size_t)max_res, C = c.channels, K = c.branches;
  const size_t max_tiles = 3 * ((size_t)max_res / 16 + 4096);
  size_t off = align256(max_tiles * sizeof(TileDesc)) + 256;           // descriptors + amax counters
  off += 2 * K * align256(R * C * act_bytes(c.dtype));
  off += K * align256(R * C * hid_bytes(c));
  return off;
}

void arena_carve(const conet_config& c, int64_t max_res, uint8_t* base, Arena& ar) {
  const size_t R = (size_t)max_res, C = c.channels;
  const int K = c.branches;
  ar.max_res = max_res;
  ar.max_tiles = 3 * ((size_t)max_res / 16 + 4096);
  size_t off = 0;
  ar.tiles = reinterpret_cast<TileDesc*>(base + off);
  off = align256(off + ar.max_tiles * sizeof(TileDesc));
  ar.amax = reinterpret_cast<unsigned*>(base + off);
  off += 256;
  for (int p = 0; p < 2; ++p)
    for (int k = 0; k < K; ++k) { ar.act[p][k] = base + off; off += align256(R * C * act_bytes(c.dtype)); }
  for (int k = 0; k < K; ++k) { ar.hid[k] = base + off; off += align256(R * C * hid_bytes(c)); }
}

// Workspace: [packed filters][FP32 vectors][activation arena]
void plan_layout(const conet_config& c, Layout& lay) {
  const int K = c.branches, L = c.blocks, C = c.channels, Ci = c.in_channels, m = c.bits_per_symbol;
  const bool ds = c.block_type == CONET_BLOCK_SEPARABLE;
  const size_t blk_pack = ds ? packed_bytes_1x1(c.dtype, C, C) : packed_bytes(c.dtype, C, C);
  size_t off = 0;
  for (int k = 0; k < K; ++k) {
    lay.w_in[k] = off; off = align256(off + packed_bytes(c.dtype, Ci, C));
    for (int l = 0; l < branch_blocks(c, k); ++l) {
      lay.w1[k][l] = off; off = align256(off + blk_pack);
      lay.w2[k][l] = off; off = align256(off + blk_pack);
      if (block_uses_mfma32(c.dtype, C) && !c.train && !ds) {
        lay.w1f[k][l] = off; off = align256(off + packed_bytes32(c.dtype, C, C));
        lay.w2f[k][l] = off; off = align256(off + packed_bytes32(c.dtype, C, C));
      } else {
        lay.w1f[k][l] = lay.w1[k][l];
        lay.w2f[k][l] = lay.w2[k][l];
      }
    }
  }
  if (c.fusion_op == CONET_FUSE_CONCAT)
    for (int l = 0; l < L; ++l) { lay.w_cat[l] = off; off = align256(off + packed_bytes_1x1(c.dtype, K * C, C)); }
  // FP32 vectors: per branch b_in, wscale_in; per (k,l): s0 o0 b1 s1 o1 b2 ws1 ws2 (and the
  // depthwise filters of separable blocks); per l gamma beta (and bc); Wh bh
  size_t nv = 0;
  for (int k = 0; k < K; ++k) {
    lay.v_bin[k] = nv; nv += C;
    lay.v_wsin[k] = nv; nv += C;
    for (int l = 0; l < branch_blocks(c, k); ++l) {
      lay.v_blk[k][l] = nv; nv += 8 * C;
      if (ds) { lay.v_dw[k][l] = nv; nv += 18 * C; }
    }
  }
  for (int l = 0; l < L; ++l) { lay.v_gamma[l] = nv; nv += C; lay.v_beta[l] = nv; nv += C; }
  if (c.fusion_op == CONET_FUSE_CONCAT)
    for (int l = 0; l < L; ++l) { lay.v_bcat[l] = nv; nv += C; }
  lay.v_wh = nv; nv += (size_t)m * C;
  lay.v_bh = nv; nv += m;
  lay.n_vec = nv;
  lay.vec = off; off = align256(off + nv * 4);
  lay.arena = off;
  off = align256(off + arena_bytes(c, c.max_res));
  if (c.train) off = align256(off + train_bytes(c, lay, off));
  lay.total = off;
}

}  // namespace conet

using namespace conet;

// ---------------------------------------------------------------- ABI
extern "C" {

const char* conet_last_error(void) { return g_last_error.c_str(); }

size_t conet_weight_count(const conet_config* cfg) {
  if (check_config(cfg) != CONET_OK) return 0;
  return n_params(*cfg);
}

size_t conet_workspace_bytes(const conet_config* cfg) {
  if (check_config(cfg) != CONET_OK) return 0;
  Layout lay;
  plan_layout(*cfg, lay);
  return lay.total;
}

conet_status conet_create(const conet_config* cfg, const float* w, size_t n_weights, void* workspace,
                          size_t workspace_bytes, conet_model** out) {
  g_last_error.clear();
  if (!out) return fail(CONET_EINVAL, "null output handle");
  *out = nullptr;
  conet_status st = check_config(cfg);
  if (st != CONET_OK) return st;
  if (!w || !workspace) return fail(CONET_EINVAL, "null weights or workspace");
  if (n_weights != n_params(*cfg)) return fail(CONET_EINVAL, "blob has %zu values, configuration needs %zu", n_weights, n_params(*cfg));
  if (cfg->norm == CONET_NORM_BN) {  // running variances must keep var + eps positive
    const size_t C = cfg->channels, L = cfg->blocks, tail = n_weights - 2 * L * C;
    for (size_t l = 0; l < L; ++l)
      for (size_t c = 0; c < C; ++c) {
        const float v = w[tail + (2 * l + 1) * C + c];
        if (!(v + cfg->ln_eps > 0.f) || !std::isfinite(v)) return fail(CONET_EINVAL, "BatchNorm variance %g of block %zu", v, l + 1);
      }
  }
  if (((uintptr_t)workspace & 255) != 0) return fail(CONET_EINVAL, "workspace must be 256-byte aligned");
  conet_model* M = new (std::nothrow) conet_model();
  if (!M) return fail(CONET_ENOMEM, "host allocation failed");
  M->cfg = *cfg;
  plan_layout(*cfg, M->lay);
  if (workspace_bytes < M->lay.total) {
    size_t need = M->lay.total;
    delete M;
    return fail(CONET_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, need);
  }
  M->ws = (uint8_t*)workspace;
  arena_carve(*cfg, cfg->max_res, M->ws + M->lay.arena, M->arena);
  hipError_t e = hipGetDevice(&M->device);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&M->n_cu, hipDeviceAttributeMultiprocessorCount, M->device);
  if (e != hipSuccess) { delete M; return hip_fail(e, "hipGetDevice"); }
  st = noalloc_setup(M->device);
  if (st != CONET_OK) { delete M; return st; }

  const int K = cfg->branches, L = cfg->blocks, C = cfg->channels, Ci = cfg->in_channels, m = cfg->bits_per_symbol;
  const Layout& lay = M->lay;
  // host image of the filter + vector regions, uploaded in one copy
  std::vector<uint8_t> img(lay.vec + lay.n_vec * 4, 0);
  float* vec = reinterpret_cast<float*>(img.data() + lay.vec);
  M->blob.assign(w, w + n_weights);
  const float* p = w;
  for (int k = 0; k < K; ++k) {
    pack_filter(cfg->dtype, Ci, C, p, img.data() + lay.w_in[k], vec + lay.v_wsin[k]);
    p += (size_t)C * Ci * 9;
    memcpy(vec + lay.v_bin[k], p, C * 4); p += C;
    for (int l = 0; l < branch_blocks(*cfg, k); ++l) {
      float* vb = vec + lay.v_blk[k][l];  // s0 o0 b1 s1 o1 b2 ws1 ws2
      if (cfg->block_type == CONET_BLOCK_SEPARABLE) {
        float* dw = vec + lay.v_dw[k][l];  // [9][C] per conv, tap-major
        for (int i = 0; i < 2; ++i) {
          // s0 o0 D1 P1 b1 | s1 o1 D2 P2 b2
          memcpy(vb + (3 * i) * C, p, C * 4); p += C;        // s0 / s1
          memcpy(vb + (3 * i + 1) * C, p, C * 4); p += C;    // o0 / o1
          // depthwise filters are conv operands: BF16 models hold them rounded to BF16
          for (int ch = 0; ch < C; ++ch)
            for (int tap = 0; tap < 9; ++tap) {
              float w = p[ch * 9 + tap];
              if (cfg->dtype == DT_BF16) {
                const uint32_t u = (uint32_t)bf16_bits(w) << 16;
                memcpy(&w, &u, 4);
              }
              dw[(size_t)i * 9 * C + tap * C + ch] = w;
            }
          p += (size_t)9 * C;
          pack_1x1(cfg->dtype, C, C, p, img.data() + (i == 0 ? lay.w1[k][l] : lay.w2[k][l]));
          p += (size_t)C * C;
          memcpy(vb + (i == 0 ? 2 : 5) * C, p, C * 4); p += C;  // b1 / b2
        }
        continue;
      }
      memcpy(vb + 0 * C, p, C * 4); p += C;                 // s0
      memcpy(vb + 1 * C, p, C * 4); p += C;                 // o0
      pack_filter(cfg->dtype, C, C, p, img.data() + lay.w1[k][l], vb + 6 * C);
      if (lay.w1f[k][l] != lay.w1[k][l]) pack_filter32(cfg->dtype, C, C, p, vb + 6 * C, img.data() + lay.w1f[k][l]);
      p += (size_t)C * C * 9;
      memcpy(vb + 2 * C, p, C * 4); p += C;                 // b1
      memcpy(vb + 3 * C, p, C * 4); p += C;                 // s1
      memcpy(vb + 4 * C, p, C * 4); p += C;                 // o1
      pack_filter(cfg->dtype, C, C, p, img.data() + lay.w2[k][l], vb + 7 * C);
      if (lay.w2f[k][l] != lay.w2[k][l]) pack_filter32(cfg->dtype, C, C, p, vb + 7 * C, img.data() + lay.w2f[k][l]);
      p += (size_t)C * C * 9;
      memcpy(vb + 5 * C, p, C * 4); p += C;                 // b2
    }
  }
  for (int l = 0; l < L; ++l) {
    memcpy(vec + lay.v_gamma[l], p, C * 4); p += C;
    memcpy(vec + lay.v_beta[l], p, C * 4); p += C;
  }
  memcpy(vec + lay.v_wh, p, (size_t)m * C * 4); p += (size_t)m * C;
  memcpy(vec + lay.v_bh, p, m * 4); p += m;
  if (cfg->fusion_op == CONET_FUSE_CONCAT)
    for (int l = 0; l < L; ++l) {
      pack_1x1(cfg->dtype, K * C, C, p, img.data() + lay.w_cat[l]);
      p += (size_t)C * K * C;
      memcpy(vec + lay.v_bcat[l], p, C * 4); p += C;
    }
  if (cfg->norm == CONET_NORM_BN) {
    // BatchNorm with running statistics is a per-channel affine: fold it into gamma/beta,
    // gamma' = gamma / sqrt(var + eps), beta' = beta - mean gamma'. A training model keeps
    // gamma and beta as given: it normalises by each batch's own statistics.
    for (int l = 0; l < L && !cfg->train; ++l) {
      const float* mean = p + (size_t)l * 2 * C;
      const float* var = mean + C;
      float* g = vec + lay.v_gamma[l];
      float* b = vec + lay.v_beta[l];
      for (int c = 0; c < C; ++c) {
        const float gs = (float)((double)g[c] / std::sqrt((double)var[c] + (double)cfg->ln_eps));
        b[c] = (float)((double)b[c] - (double)mean[c] * (double)gs);
        g[c] = gs;
      }
    }
    p += (size_t)2 * L * C;
  }
  e = hipMemcpy(M->ws, img.data(), img.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { delete M; return hip_fail(e, "upload of packed weights"); }
  M->act_scales.assign(1 + 2 * K * L, 1.0f);
  M->scales_set = false;
  if (cfg->train) blob_offsets(*cfg, M->bo);
  if (cfg->train) {
    conet_status st = train_init(M);
    if (st != CONET_OK) { delete M; return st; }
  }
  *out = M;
  return CONET_OK;
}

conet_status conet_destroy(conet_model* M) {
  if (!M) return fail(CONET_EINVAL, "null model");
  delete M;
  return CONET_OK;
}

conet_status conet_set_act_scales(conet_model* M, const float* s, size_t n) {
  if (!M || !s) return fail(CONET_EINVAL, "null argument");
  if (M->cfg.dtype != DT_FP8) return fail(CONET_EINVAL, "activation scales apply to FP8 models only");
  if (n != M->act_scales.size()) return fail(CONET_EINVAL, "expected %zu scales, got %zu", M->act_scales.size(), n);
  for (size_t i = 0; i < n; ++i)
    if (!(s[i] > 0.f) || !std::isfinite(s[i])) return fail(CONET_EINVAL, "scale %zu is not a positive finite number", i);
  M->act_scales.assign(s, s + n);
  M->scales_set = true;
  return CONET_OK;
}

conet_status conet_get_act_scales(conet_model* M, float* s, size_t n) {
  if (!M || !s) return fail(CONET_EINVAL, "null argument");
  if (n != M->act_scales.size()) return fail(CONET_EINVAL, "expected %zu scales, got %zu", M->act_scales.size(), n);
  std::copy(M->act_scales.begin(), M->act_scales.end(), s);
  return CONET_OK;
}

conet_status conet_forward(conet_model* M, const float* x, int32_t B, int32_t T, int32_t F, float* llr,
                           int32_t save, void* stream) {
  if (!M) return fail(CONET_EINVAL, "null model");
  if (save && !M->cfg.train) return fail(CONET_ESTATE, "save_for_backward needs a model created with train = 1");
  if (B == 0) return CONET_OK;
  if (!x || !llr) return fail(CONET_EINVAL, "null tensor pointer");
  if (B < 0 || T < 1 || T > TMAX || F < 1) return fail(CONET_ESHAPE, "bad shape B=%d T=%d F=%d (need T in 1..14)", B, T, F);
  if ((int64_t)B * T * F > M->cfg.max_res) return fail(CONET_ESHAPE, "B*T*F = %lld exceeds max_res %lld", (long long)B * T * F, (long long)M->cfg.max_res);
  if (M->cfg.dtype == DT_FP8 && !M->scales_set) return fail(CONET_ESTATE, "FP8 model needs activation scales (set or calibrate)");
  Geometry geo;
  geo.uniform = true; geo.B = B; geo.T = T; geo.F = F;
  if (save) {
    conet_status st = run_forward(M, M->train_arena, x, geo, llr, (hipStream_t)stream, nullptr, nullptr, true);
    M->saved = st == CONET_OK;
    M->saved_B = B; M->saved_T = T; M->saved_F = F;
    M->saved_x = x;
    return st;
  }
  return run_forward(M, M->arena, x, geo, llr, (hipStream_t)stream, nullptr);
}

conet_status conet_forward_grid(conet_model* M, const float* y, int32_t B, int32_t T, int32_t F, int32_t n_rx,
                                float* llr, void* stream) {
  if (!M) return fail(CONET_EINVAL, "null model");
  if (B == 0) return CONET_OK;
  if (!y || !llr) return fail(CONET_EINVAL, "null tensor pointer");
  if (B < 0 || T <= PILOT_T1 || T > TMAX || F < 1)
    return fail(CONET_ESHAPE, "bad shape B=%d T=%d F=%d (need 12 <= T <= 14: both pilot symbols)", B, T, F);
  if (n_rx < 1 || 4 * n_rx > M->cfg.in_channels)
    return fail(CONET_ESHAPE, "n_rx = %d needs 4 n_rx <= C_in = %d", n_rx, M->cfg.in_channels);
  if ((int64_t)B * T * F > M->cfg.max_res) return fail(CONET_ESHAPE, "B*T*F = %lld exceeds max_res %lld", (long long)B * T * F, (long long)M->cfg.max_res);
  if (M->cfg.dtype == DT_FP8 && !M->scales_set) return fail(CONET_ESTATE, "FP8 model needs activation scales (set or calibrate)");
  Geometry geo;
  geo.uniform = true; geo.B = B; geo.T = T; geo.F = F; geo.grid_rx = n_rx;
  return run_forward(M, M->arena, y, geo, llr, (hipStream_t)stream, nullptr);
}

conet_status conet_forward_ragged(conet_model* M, const float* x, int32_t n_slots, int32_t T, const int32_t* F_host,
                                  float* llr, void* stream) {
  if (!M) return fail(CONET_EINVAL, "null model");
  if (n_slots == 0) return CONET_OK;
  if (!x || !llr || !F_host) return fail(CONET_EINVAL, "null pointer");
  if (n_slots < 0 || T < 1 || T > TMAX) return fail(CONET_ESHAPE, "bad shape n_slots=%d T=%d", n_slots, T);
  int64_t total = 0;
  for (int s = 0; s < n_slots; ++s) {
    if (F_host[s] < 1) return fail(CONET_ESHAPE, "slot %d has F=%d", s, F_host[s]);
    total += (int64_t)T * F_host[s];
  }
  if (total > M->cfg.max_res) return fail(CONET_ESHAPE, "ragged batch has %lld REs, max_res is %lld", (long long)total, (long long)M->cfg.max_res);
  if (M->cfg.dtype == DT_FP8 && !M->scales_set) return fail(CONET_ESTATE, "FP8 model needs activation scales (set or calibrate)");
  Geometry geo;
  geo.uniform = false; geo.T = T; geo.n_slots = n_slots; geo.F_host = F_host;
  return run_forward(M, M->arena, x, geo, llr, (hipStream_t)stream, nullptr);
}

}  // extern "C"

extern "C" int32_t conet_block_tile_width(const conet_model* M) {
  return M ? block_tile_width(M->cfg.dtype, M->cfg.channels, M->cfg.branches, TW_WIDE, M->cfg.train != 0) : 0;
}
