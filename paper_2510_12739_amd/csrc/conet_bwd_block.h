// Declarations of the fused input-gradient block (conet_bwd_block.hip), used by the backward
// launch sequence (conet_backward.hip).
#pragma once
#include "conet_kernels.h"

namespace conet {

// Input gradient of one residual block in one launch (the adjoint of the fused forward block):
//   dc1 = s1 [h > 0] convT2(dO)               (stored: the filter gradient of conv 1 reads it)
//   dx  = dO + s0 [s0 x + o0 > 0] convT1(dc1)  (masked by [x > 0] when mask_out)
// with dc1 kept in LDS for its own tile's second transposed conv. Each (work-group, wave)
// writes one row of partial sums: [rows) holds sum dz1 (h - o1) / s1 and sum dz1, [rows,
// 2 rows) holds sum dz0 x and sum dz0 (zero for an MRB, s0 = null), each row 3 * C floats.
struct BwdBlockArgs {
  const void* dO[KMAX_ARGS];       // gradient of the block output, [RE][C] Act
  const void* h[KMAX_ARGS];        // conv 1's activation h saved by the forward
  const void* x[KMAX_ARGS];        // block input x saved by the forward
  const void* wt1[KMAX_ARGS];      // fragment-packed transposed filters of conv 1 and conv 2
  const void* wt2[KMAX_ARGS];
  const float* s1[KMAX_ARGS];      // affine after conv 1
  const float* o1[KMAX_ARGS];
  const float* s0[KMAX_ARGS];      // pre-activation affine; null => ReLU only (MRB)
  const float* o0[KMAX_ARGS];
  void* dc1[KMAX_ARGS];            // out: [RE][C] Act
  void* dx[KMAX_ARGS];             // out: [RE][C] Act
  float* part[KMAX_ARGS];          // out: 2 * rows partial rows of 3 * C floats
  int rows;                        // n_tiles * CONV_NW
  int mask_out;                    // the block input is the input layer's ReLU output
  int T, F, tiles_per_slot, tw;    // tw: set by the launcher
  const TileDesc* tiles;           // always null (whole slots)
};
// Output subcarriers per tile of the fused input-gradient block (0: none for this dtype / C;
// the backward then runs the two transposed convs as separate launches).
int bwd_block_tile_width(int dtype, int C);
hipError_t launch_bwd_block(int dtype, int C, BwdBlockArgs& a, int n_tiles, int grid_y, hipStream_t s);

}  // namespace conet
