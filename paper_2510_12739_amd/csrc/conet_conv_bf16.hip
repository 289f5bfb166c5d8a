// BF16 instantiations of the 3x3 conv kernels and the fused block kernel (one
// translation unit per dtype).
#include "conet_block_impl.h"

namespace conet {

hipError_t launch_conv_bf16(int mode, int cin, int cout, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  return launch_dtype<ArithBF16>(mode, cin, cout, a, n_tiles, grid_y, s);
}

int conv_tile_width_bf16(int cin, int cout) { return tile_width_dtype<ArithBF16>(cin, cout); }

hipError_t launch_block_bf16(int kind, bool narrow, int C, BlockArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  return launch_block_dtype<ArithBF16>(kind, narrow, C, a, n_tiles, grid_y, s);
}

int block_tile_width_bf16(int C, bool narrow) { return block_tile_width_dtype<ArithBF16>(C, narrow); }

}  // namespace conet
