// BF16 instantiations of the 3x3 conv kernels and the fused block kernels (one
// translation unit per dtype).
#include "conet_block32_impl.h"

namespace conet {

hipError_t launch_conv_bf16(int mode, int cin, int cout, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  return launch_dtype<ArithBF16>(mode, cin, cout, a, n_tiles, grid_y, s);
}

int conv_tile_width_bf16(int cin, int cout) { return tile_width_dtype<ArithBF16>(cin, cout); }
int conv_tile_width_narrow_bf16(int cin, int cout) { return tile_width_narrow_dtype<ArithBF16>(cin, cout); }

// 96 channels: the 32x32x16 kernel (its own filter packing); 16, 32, 64: the 16x16x32 one.
hipError_t launch_block_bf16(int kind, int wclass, int C, BlockArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  if (C == B32_C) {
    if (wclass == TW_NARROW3) return hipErrorInvalidValue;
    return launch_block32<Mfma32BF16<>>(kind, a, n_tiles, grid_y, s);
  }
  return launch_block_dtype<ArithBF16>(kind, wclass, C, a, n_tiles, grid_y, s);
}

int block_tile_width_bf16(int C, int wclass) {
  if (C == B32_C) return wclass == TW_NARROW3 ? 0 : Mfma32BF16<>::TWO;
  return block_tile_width_dtype<ArithBF16>(C, wclass);
}

}  // namespace conet
