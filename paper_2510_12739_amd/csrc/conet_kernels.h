// Internal interface between the C-ABI host code and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace conet {

enum { DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2 };
constexpr int KMAX_ARGS = 8;
constexpr int CONV_NW = 4;  // waves per work-group of the conv kernels

struct TileDesc;

// Arguments of one conv launch. Per-branch arrays are indexed by the work-group's
// branch, blockIdx.y + k_off. Activation tensors are [RE][channels].
struct ConvArgs {
  const void* in[KMAX_ARGS];       // conv input (mode 0: FP32 features)
  const void* resid[KMAX_ARGS];    // block input x for the residual add (modes 2, 3)
  void* out[KMAX_ARGS];            // output tensor (nullable)
  const void* sup[KMAX_ARGS];      // mode 4: this block's stored support-branch outputs
  const void* wpack[KMAX_ARGS];    // fragment-packed filters
  const float* bias[KMAX_ARGS];
  const float* pre_s[KMAX_ARGS];   // mode 1 prologue affine; null => ReLU only (MRB)
  const float* pre_o[KMAX_ARGS];
  const float* post_s[KMAX_ARGS];  // mode 1 epilogue affine
  const float* post_o[KMAX_ARGS];
  const float* wscale[KMAX_ARGS];  // FP8: per-output-channel filter scales
  float in_qscale[KMAX_ARGS];      // FP8: 1 / s_a of this conv's input operand
  float deq[KMAX_ARGS];            // FP8: s_a of this conv's input operand
  float out_qscale[KMAX_ARGS];     // FP8: 1 / s_a of the consumer of this output (mode 1)
  const float* gamma;              // mode 4 LayerNorm affine
  const float* beta;
  const float* Wh;                 // head [m][C] (null-free when llr is set)
  const float* bh;
  float* llr;                      // [RE][m] FP32, or null
  int m;
  int K;                           // branches (mode 4 multiplies sup[1..K-1])
  int k_off;                       // branch of blockIdx.y == 0
  float eps;
  // geometry
  int T, F;                        // uniform batches: every slot T x F
  int tiles_per_slot;
  int tw;                          // subcarriers per tile (set by the launcher)
  const TileDesc* tiles;           // ragged batches: one descriptor per tile, else null
  unsigned* amax;                  // mode 1 calibration: per-branch max |output| (no store)
  // backward (modes 5, 6)
  const void* aux[KMAX_ARGS];      // mode 5: the block's saved h; mode 6: the block's saved input x
  float* part[KMAX_ARGS];          // per-wave per-channel partial sums [gridDim.x * waves][NPART][C]
  int mask_out;                    // mode 6: store dx * (x > 0) (input-layer ReLU adjoint)
  void* save_o0;                   // mode 4 (training): also store the main output before fusion
  int inner_branches;              // mode 0: run branches k_off .. k_off + n - 1 in every work-group
                                   // (one staged feature tile; launch with grid.y = 1)
  int grid_rx;                     // mode 0: > 0 => in[] is the received grid, FP32 [RE][grid_rx][2],
                                   // and the features are formed while staging (LS + interpolation)
  int narrow;                      // modes 0-4, FP32: 1 => the narrow tile width of
                                   // conv_tile_width_narrow (a batch too small to fill the GPU)
  int fusion_sum;                  // mode 4: fuse by addition instead of the product
  int norm_affine;                 // mode 4: gamma/beta are a per-channel affine (BatchNorm with
                                   // running statistics folded in) instead of LayerNorm's
  int feedback;                    // mode 4: also rewrite sup[k] <- sup[k] + fused output (Example II)
};

// Subcarriers per tile used for a (dtype, C_in, C_out) conv.
int conv_tile_width(int dtype, int cin, int cout);
// The width with ConvArgs::narrow set: 16 for FP32 convs whose default is wider (more, shorter
// work-groups for a batch whose tiles cannot fill the GPU), else the default.
int conv_tile_width_narrow(int dtype, int cin, int cout);
bool conv_supported(int dtype, int cin, int cout);
// mode: 0 input layer, 1 block conv 1, 2 block conv 2 (+ residual, + head on branch 0
// if llr is set), 4 block conv 2 of the main net + product with the stored support
// outputs + LayerNorm (+ head); backward input-gradient convs (flipped, transposed
// filters): 5 through the block's second conv (-> d of the first conv's output), 6
// through its first conv (-> d of the block input). Branch: blockIdx.y + k_off.
hipError_t launch_conv(int dtype, int mode, int cin, int cout, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s);

// ---------------------------------------------------------------- fused residual block
// Both convs of one block (per branch blockIdx.y + k_off) in one launch, h kept in LDS:
// out = x + conv2(ReLU(s1 (conv1(pre(x)) + b1) + o1)) + b2; with `main`, the main branch
// of a fused block (product with sup[1..K-1], LayerNorm, head when llr is set).
struct BlockArgs {
  const void* x[KMAX_ARGS];        // block input (residual stream), [RE][C] Act
  void* out[KMAX_ARGS];            // block output (nullable); main: out[0]
  const void* sup[KMAX_ARGS];      // main: this block's stored support-branch outputs
  const void* w1[KMAX_ARGS];       // fragment-packed filters of conv 1 and conv 2
  const void* w2[KMAX_ARGS];
  const float* b1[KMAX_ARGS];
  const float* b2[KMAX_ARGS];
  const float* pre_s[KMAX_ARGS];   // pre-activation affine; null => ReLU only (MRB)
  const float* pre_o[KMAX_ARGS];
  const float* post_s[KMAX_ARGS];  // affine after conv 1
  const float* post_o[KMAX_ARGS];
  const float* ws1[KMAX_ARGS];     // FP8: per-output-channel filter scales
  const float* ws2[KMAX_ARGS];
  float q1[KMAX_ARGS], deq1[KMAX_ARGS];  // FP8: 1 / s and s of conv 1's operand pre(x)
  float q2[KMAX_ARGS], deq2[KMAX_ARGS];  // FP8: 1 / s and s of conv 2's operand h
  const float* gamma;
  const float* beta;
  const float* Wh;
  const float* bh;
  float* llr;                      // [RE][m] FP32, or null
  int m, K, k_off;
  float eps;
  int T, F, tiles_per_slot, tw;    // tw: set by the launcher
  const TileDesc* tiles;           // ragged batches, else null
  int fusion_sum;                  // main: fuse by addition instead of the product
  int norm_affine;                 // main: per-channel affine (folded BatchNorm) instead of LayerNorm
  int feedback;                    // main: also rewrite sup[k] <- sup[k] + fused output (Example II)
  // training forward (nullable): h of branch k as stored by the two-conv path, and the
  // main branch's output before the fusion (or branch 0's output before the head)
  void* hid_out[KMAX_ARGS];
  void* save_o0;
};
// Output subcarriers per fused tile; 0 when (dtype, C, K) runs as two conv launches, or when
// there is no kernel of that width class. TW_WIDE: batches that fill the GPU; TW_NARROW: a
// batch whose wide tiles cannot fill it once; TW_NARROW3: such a batch whose paired launches
// would need two rounds of narrow work-groups at two per CU (built for three per CU). train:
// the model keeps training state (its forward must read the filter packs the optimiser updates).
enum { TW_WIDE = 0, TW_NARROW = 1, TW_NARROW3 = 2 };
constexpr int BLOCK_KMAX = 4;  // fused main-branch kernels exist for K <= 4
// FP8 and BF16 at 96 channels run the fused block on the 32x32 MFMAs, which read filters in
// their own fragment packing (pack_filter32). Training models do not use them (the
// optimiser regenerates only the 16x16 packs).
inline bool block_uses_mfma32(int dtype, int C) { return C == 96 && (dtype == DT_FP8 || dtype == DT_BF16); }
int block_tile_width(int dtype, int C, int K, int wclass, bool train = false);
// kind BLOCK_PLAIN: branches blockIdx.y + k_off, no fusion epilogue (support branches, or
// every branch of a block without fusion; head on branch 0 when llr is set); BLOCK_MAIN: the
// main branch of a fused block (k_off = 0, grid.y = 1); BLOCK_PAIR: grid.y = K, blockIdx.y 0
// is the main branch of block l and 1..K-1 the support branches of block l + 1 (no head).
enum { BLOCK_PLAIN = 0, BLOCK_MAIN = 1, BLOCK_PAIR = 2 };
hipError_t launch_block(int dtype, int kind, int wclass, int C, BlockArgs& a, int n_tiles, int grid_y, hipStream_t s);

// ---------------------------------------------------------------- block and fusion variants
// Depthwise-separable residual block (both separable convs in one launch, h in LDS), per
// branch blockIdx.y + k_off: out = x + P2 dw2(ReLU(s1 (P1 dw1(pre(x)) + b1) + o1)) + b2, on
// tiles of DS_TW subcarriers.
constexpr int DS_TW = 16;
struct DsArgs {
  const void* x[KMAX_ARGS];        // block input [RE][C] Act
  void* out[KMAX_ARGS];            // block output [RE][C]: Act, or FP32 where out_f32[k]
  int out_f32[KMAX_ARGS];
  const float* pre_s[KMAX_ARGS];   // pre-activation affine; null => ReLU only (MRB)
  const float* pre_o[KMAX_ARGS];
  const float* dw1[KMAX_ARGS];     // depthwise filters, FP32 [tap = 3 (dt + 1) + df + 1][C]
  const float* dw2[KMAX_ARGS];
  const void* pw1[KMAX_ARGS];      // 1x1 filters in pack_1x1 order
  const void* pw2[KMAX_ARGS];
  const float* b1[KMAX_ARGS];
  const float* b2[KMAX_ARGS];
  const float* post_s[KMAX_ARGS];  // affine after the first separable conv
  const float* post_o[KMAX_ARGS];
  int k_off;
  int T, F, tiles_per_slot, tw;    // tw: set by the launcher
  const TileDesc* tiles;           // ragged batches, else null
};
bool ds_supported(int dtype, int C);
hipError_t launch_ds_block(int dtype, int C, DsArgs& a, int n_tiles, int grid_y, hipStream_t s);

// Per-RE fusion epilogue over stored block outputs: P = main (EPI_NONE), main * prod sup[k]
// (EPI_PRODUCT), main + sum sup[k] (EPI_SUM) or Wc [main; sup[1]; ..] + bc (EPI_CONCAT, MFMA);
// then LayerNorm (gamma, beta) or the affine gamma P + beta (norm_affine) -- none for
// EPI_NONE -- giving A; A is stored to `out` (nullable), added into every sup[k] with
// feedback, and fed to the head when llr is set.
enum { EPI_NONE = 0, EPI_PRODUCT = 1, EPI_SUM = 2, EPI_CONCAT = 3 };
struct FuseArgs {
  const void* main;                // [RE][C] FP32 (main_f32) or Act
  int main_f32;
  void* sup[KMAX_ARGS];            // k = 1..K-1: stored support outputs [RE][C] Act
  int K;
  const void* wcat;                // EPI_CONCAT: Wc in pack_1x1 order (C x K C)
  const float* bcat;
  const float* gamma;
  const float* beta;
  int norm_affine;
  float eps;
  void* out;                       // A [RE][C] Act, or null
  int feedback;
  const float* Wh;
  const float* bh;
  float* llr;                      // [RE][m] FP32, or null
  int m;
  int64_t n_re;
};
bool concat_supported(int dtype, int C, int K);
hipError_t launch_fuse_epilogue(int dtype, int C, int mode, FuseArgs& a, hipStream_t s);

// ---------------------------------------------------------------- training kernels
// Filter gradient of a 3x3 conv over a batch: dW[o][tap*CIN + ch] = sum_re dOut[re][o] *
// In[re shifted by tap][ch] (In optionally through the block's pre-activation), and
// db[o] = sum_re dOut[re][o]. Each work-group accumulates over its share of tiles and
// writes one partial row; the sum over rows happens in reduce_launch (fixed order).
struct WgradArgs {
  const void* dout[KMAX_ARGS];     // [RE][COUT] Act
  const void* in[KMAX_ARGS];       // [RE][CIN] Act, or FP32 features (input layer)
  const float* pre_s[KMAX_ARGS];   // prologue on In: affine + ReLU; null with relu => ReLU only
  const float* pre_o[KMAX_ARGS];
  int prologue;                    // 0 none, 1 per-branch (affine if pre_s else ReLU)
  float* part_w[KMAX_ARGS];        // [gridDim.x][COUT][9 * CIN]
  float* part_b[KMAX_ARGS];        // [gridDim.x][COUT]
  int T, F, tiles_per_slot, n_tiles, tw;
  int grid;                        // work-groups per branch (wgrad_grid), one partial row each
};
int wgrad_tile_width(int dtype);
// Work-groups per branch of a filter-gradient launch over `branches` branches: one round of one
// work-group per CU over all branches (each loops over its share of the tiles), at most 256.
int wgrad_grid(int n_tiles, int branches, int n_cu);
hipError_t launch_wgrad(int dtype, bool in_f32, int cin, int cout, WgradArgs& a, int grid_y, hipStream_t s);

// Head / LayerNorm / product adjoint of one block (or the head alone after an unfused
// last block). One thread per (RE, 16-channel quarter).
struct FuseBwdArgs {
  const float* dllr;               // [RE][m] (last block) or null
  const void* dA;                  // [RE][C] gradient of the fused main activation (other blocks)
  const void* O[KMAX_ARGS];        // block outputs: O[0] saved before fusion, O[k>0] stored supports
  const void* dnext[KMAX_ARGS];    // k>0: gradients of the next block's support inputs (or null)
  void* dO[KMAX_ARGS];             // out: gradients of the block outputs
  const float* gamma;
  const float* beta;
  const float* Wh;                 // [m][C]
  int m, K, C, fused, head;
  float eps;
  int64_t n_re;
  float* part;                     // [gridDim.x][NP] partial sums: dgamma C, dbeta C, dWh m*C, dbh m
  // BatchNorm by batch statistics (bn_mu non-null): per-channel mean and 1/sqrt(var + eps) of
  // the forward. The adjoint needs the batch sums of dA and dA ahat, which are the gamma and
  // beta gradients: pass 1 forms them (partial sums only, no dO), pass 2 reads them back
  // (bn_dgamma, bn_dbeta, already reduced) and writes dO
  const float* bn_mu;
  const float* bn_rs;
  const float* bn_dgamma;
  const float* bn_dbeta;
  int bn_pass;
  void* a_out;                     // head launch: [RE][C] the head's input A (compute dtype), or null
};
hipError_t launch_fuse_bwd(int dtype, FuseBwdArgs& a, int grid, hipStream_t s);

// Head weight gradient from the stored head input: part[row][col0 + j C + c] = this row's share
// of sum_re dllr[re][j] A[re][c] (one row per work-group, row stride ld floats).
struct HeadWgradArgs {
  const void* A;                   // [RE][C] compute dtype
  const float* dllr;               // [RE][m]
  int m;
  int64_t n_re;
  float* part;
  int ld, col0;
};
hipError_t launch_head_wgrad(int dtype, int C, HeadWgradArgs& a, int grid, hipStream_t s);

// BatchNorm statistics of the product P = O_0 O_1 ... O_{K-1} over every RE of a batch, per
// channel. Pass 0: work-group partial sums of P; pass 1: of (P - mean)^2 (mean from pass 0).
struct BnStatsArgs {
  const void* main;                // [RE][C] O_0 as stored (compute dtype)
  const void* sup[KMAX_ARGS];      // [RE][C] O_k, k >= 1
  int K, C, pass;
  int64_t n_re;
  const float* mean;               // pass 1: the batch mean
  float* part;                     // [gridDim.x][C]
};
// Sums the partials in a fixed order. Pass 0 writes the mean; pass 1 writes 1/sqrt(var + eps),
// the folded scale gamma / sqrt(var + eps) and shift beta - mean scale, and, if running_mean is
// non-null, moves the running statistics by `momentum` towards the batch's (the variance
// unbiased, n / (n - 1)).
struct BnFinishArgs {
  const float* part;
  int groups, C, pass;
  int64_t n_re;
  float eps, momentum;
  const float* gamma;
  const float* beta;
  float* mean;                     // [C]
  float* rs;                       // [C]
  float* scale;                    // [C]
  float* shift;                    // [C]
  float* running_mean;             // [C] or null
  float* running_var;              // [C]
};
int bn_stats_grid(int64_t n_re);
hipError_t launch_bn_stats(int dtype, BnStatsArgs& a, int grid, hipStream_t s);
hipError_t launch_bn_finish(BnFinishArgs& a, hipStream_t s);

// Sum of `rows` rows of `cols` floats (row stride `ld`) into dst[map(j)], in a fixed
// order: stage 1 sums chunks of 256 rows into tmp[chunk][cols], stage 2 sums the chunks.
// map: 0 identity; 1 filter: j = o*(9*cin) + tap*cin + ch -> ((o*cin + ch)*9 + tap).
struct ReduceSeg {
  const float* src;
  float* dst;
  int rows, cols, ld, map, cin;
  float* tmp;                      // [ceil(rows / 256)][cols] (set by the host)
};
constexpr int REDUCE_CHUNK = 256;
hipError_t launch_reduce(const ReduceSeg* segs_dev, int n_segs, int max_cols, int max_chunks, hipStream_t s);

hipError_t launch_bce(const float* llr, const uint8_t* bits, const uint8_t* data_mask, int64_t n_re, int T, int F,
                      int m, float inv_count, float* dllr, float* part, int grid, hipStream_t s);
hipError_t launch_adam(float* w, const float* g, float* mo, float* ve, int64_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2, hipStream_t s);
hipError_t launch_repack(const float* master, const int32_t* map, void* dst, int64_t n, int dtype, hipStream_t s);
hipError_t launch_gather(const float* master, const int32_t* map, float* dst, int64_t n, hipStream_t s);
hipError_t launch_sum(const float* x, int n, float* out, hipStream_t s);

}  // namespace conet
