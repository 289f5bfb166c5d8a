// Internal interface between the C-ABI host code and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace conet {

enum { DT_F32 = 0, DT_BF16 = 1, DT_FP8 = 2, DT_F64 = 3 };
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
};

// Subcarriers per tile used for a (dtype, C_in, C_out) conv.
int conv_tile_width(int dtype, int cin, int cout);
bool conv_supported(int dtype, int cin, int cout);
// mode: 0 input layer, 1 block conv 1, 2 block conv 2 (+ residual, + head on branch 0
// if llr is set), 4 block conv 2 of the main net + product with the stored support
// outputs + LayerNorm (+ head). Branch of a work-group: blockIdx.y + k_off.
hipError_t launch_conv(int dtype, int mode, int cin, int cout, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s);

}  // namespace conet
