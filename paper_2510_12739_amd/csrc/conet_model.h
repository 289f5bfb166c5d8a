// Host-side model state of the CoNet-Rx library.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "conet.h"
#include "conet_common.h"
#include "conet_kernels.h"

namespace conet {

constexpr int LMAX = 32;

// Byte offsets into the caller's workspace (vector offsets are in floats from `vec`).
struct Layout {
  size_t w_in[KMAX_ARGS];
  size_t w1[KMAX_ARGS][LMAX], w2[KMAX_ARGS][LMAX];
  size_t w1f[KMAX_ARGS][LMAX], w2f[KMAX_ARGS][LMAX];  // packs the fused block kernel reads
  size_t vec;                      // FP32 vectors
  size_t n_vec;
  size_t v_bin[KMAX_ARGS], v_wsin[KMAX_ARGS];
  size_t v_blk[KMAX_ARGS][LMAX];   // s0 o0 b1 s1 o1 b2 ws1 ws2 (8 C each)
  size_t v_gamma[LMAX], v_beta[LMAX], v_wh, v_bh;
  size_t v_dw[KMAX_ARGS][LMAX];    // separable blocks: depthwise filters dw1, dw2 ([9][C] each)
  size_t w_cat[LMAX], v_bcat[LMAX];  // fusion by concatenation: packed Wc_l, bc_l
  size_t arena;                    // activation arena (see Arena)
  // training (cfg.train): FP32 master, gradients, Adam moments, input-gradient filter
  // packs, index maps for regenerating packs from the master, scratch, saved levels
  size_t tr_master, tr_grad, tr_m, tr_v, tr_zero;
  size_t tr_wt1[KMAX_ARGS][LMAX], tr_wt2[KMAX_ARGS][LMAX], tr_wt_begin, tr_wt_end;
  size_t tr_map_fwd, tr_map_bwd, tr_map_vec;
  size_t tr_part_conv, tr_part_conv_rows, tr_part_w, tr_part_b, tr_part_fuse, tr_part_bce, tr_loss, tr_segs;
  size_t tr_red_tmp, tr_red_tmp_floats;
  size_t tr_levels, tr_levels_bytes;
  // BatchNorm by batch statistics (norm = CONET_NORM_BN in a training model): per block,
  // mean, 1/sqrt(var + eps), and the folded scale and shift (4 C floats), plus the
  // work-groups' partial sums of one statistics pass
  size_t tr_bn, tr_bn_part;
  size_t total;
};

// Blob offsets (in floats) of every parameter tensor.
struct BlobOffsets {
  size_t w_in[KMAX_ARGS], b_in[KMAX_ARGS];
  size_t s0[KMAX_ARGS][LMAX], o0[KMAX_ARGS][LMAX], w1[KMAX_ARGS][LMAX], b1[KMAX_ARGS][LMAX];
  size_t s1[KMAX_ARGS][LMAX], o1[KMAX_ARGS][LMAX], w2[KMAX_ARGS][LMAX], b2[KMAX_ARGS][LMAX];
  size_t gamma[LMAX], beta[LMAX], wh, bh, n;
  size_t bn_mean[LMAX], bn_var[LMAX];  // BatchNorm running statistics (norm = CONET_NORM_BN)
};

// Activation buffers of one forward in flight (the model's own, or a serving lane's).
struct Arena {
  void* act[2][KMAX_ARGS] = {};    // residual stream, ping-pong, [RE][C]
  void* hid[KMAX_ARGS] = {};       // middle activation of a block
  TileDesc* tiles = nullptr;       // ragged-batch tile descriptors
  size_t max_tiles = 0;
  int64_t max_res = 0;             // REs the buffers hold
  unsigned* amax = nullptr;        // 64 calibration counters
  // training: one buffer per level instead of ping-pong, plus backward buffers
  bool levels = false;
  void* lvl_act[LMAX + 1][KMAX_ARGS] = {};  // level l = input of block l (l = 0: input-layer output)
  void* lvl_hid[LMAX][KMAX_ARGS] = {};
  void* lvl_o0[LMAX] = {};                   // main output of block l before fusion
  void* g_dO[KMAX_ARGS] = {};
  void* g_dc1[KMAX_ARGS] = {};
  void* g_dx[2][KMAX_ARGS] = {};
};

struct Geometry {
  bool uniform = true;
  int B = 0, T = 0, F = 0;                 // uniform
  int n_slots = 0;                         // ragged
  const int32_t* F_host = nullptr;
  // ragged: pinned host staging for the tile list (capacity in descriptors), so that its
  // upload is an asynchronous copy; null: a pageable copy
  TileDesc* tiles_pin = nullptr;
  size_t tiles_pin_cap = 0;
  int grid_rx = 0;                         // > 0: x is the received grid [RE][grid_rx][2] (FP32)
};

}  // namespace conet

struct conet_model {
  conet_config cfg;
  conet::Layout lay;
  uint8_t* ws = nullptr;
  int device = 0;
  int n_cu = 256;                    // compute units of `device`
  std::vector<float> blob;           // FP32 parameters as given
  std::vector<float> act_scales;     // FP8 static activation scales
  bool scales_set = false;
  conet::Arena arena;                // activation buffers inside the workspace
  conet::Arena train_arena;          // per-level buffers (train mode)
  conet::BlobOffsets bo;
  bool saved = false;                // a forward with save_for_backward is available
  int64_t saved_B = 0;
  int saved_T = 0, saved_F = 0;
  int adam_steps = 0;
  const float* saved_x = nullptr;    // features of the saved forward (caller keeps them alive)
};

namespace conet {

conet_status fail(conet_status st, const char* fmt, ...);
conet_status hip_fail(hipError_t e, const char* what);

// Calibration hooks: when `amax` is non-null, run_forward stops after recording the
// max |operand| of every conv input, in network order, into amax_host (FP8 models).
// events (optional, 3L+2 entries): recorded on the stream before every stage and after
// the last one, so stage i took elapsed(events[i], events[i+1]). units (optional, 3L+1
// zero-initialised entries) receives per stage the conv-branch executions it ran (one
// conv of one branch over the batch; a fused block counts two).
conet_status run_forward(conet_model* M, const Arena& ar, const float* x, const Geometry& geo, float* llr,
                         hipStream_t s, std::vector<float>* calib, hipEvent_t* events = nullptr, bool save = false,
                         int32_t* units = nullptr);

size_t align256(size_t x);
size_t n_params(const conet_config& c);
size_t act_bytes_of(int dtype);
void blob_offsets(const conet_config& c, BlobOffsets& bo);
size_t train_bytes(const conet_config& c, Layout& lay, size_t base);
conet_status train_init(conet_model* M);
void pack_filter(int dtype, int cin, int cout, const float* W, uint8_t* dst, float* wscale);
size_t packed_bytes(int dtype, int cin, int cout);
void pack_filter32(int dtype, int cin, int cout, const float* W, const float* wscale, uint8_t* dst);
size_t packed_bytes32(int dtype, int cin, int cout);
void pack_1x1(int dtype, int cin, int cout, const float* W, uint8_t* dst);
size_t packed_bytes_1x1(int dtype, int cin, int cout);
uint16_t bf16_bits(float v);
// blocks of branch k: L for the main branch, support_blocks (0 => L) for the others
inline int support_depth(const conet_config& c) { return c.support_blocks > 0 ? c.support_blocks : c.blocks; }
inline int branch_blocks(const conet_config& c, int k) { return k == 0 ? c.blocks : support_depth(c); }

// Bytes of activation buffers (plus descriptor capacity) for `max_res` REs.
size_t arena_bytes(const conet_config& c, int64_t max_res);
// Carve an Arena out of `base` (256-byte aligned, arena_bytes long).
void arena_carve(const conet_config& c, int64_t max_res, uint8_t* base, Arena& ar);

// Record the address of the static scratch array of conet_forward_noalloc on `device`
// (the current device); called once per device from conet_create.
conet_status noalloc_setup(int device);

hipError_t launch_amax(const void* x, int act_dtype_bytes, int64_t n_re, int C, const float* s0, const float* o0,
                       int prologue, unsigned* out, hipStream_t s);

}  // namespace conet
