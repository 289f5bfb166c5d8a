// FP8 instantiations of the 3x3 conv kernels and the fused block kernel (one
// translation unit per dtype).
#include "conet_block32_impl.h"

namespace conet {

hipError_t launch_conv_fp8(int mode, int cin, int cout, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  return launch_dtype<ArithFP8>(mode, cin, cout, a, n_tiles, grid_y, s);
}

int conv_tile_width_fp8(int cin, int cout) { return tile_width_dtype<ArithFP8>(cin, cout); }
int conv_tile_width_narrow_fp8(int cin, int cout) { return tile_width_narrow_dtype<ArithFP8>(cin, cout); }

// 96 channels: the 32x32x64 kernel (its own filter packing); no other width is fused in FP8.
hipError_t launch_block_fp8(int kind, int wclass, int C, BlockArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  if (C != B32_C || wclass == TW_NARROW3) return hipErrorInvalidValue;
  return launch_block32<Mfma32FP8>(kind, a, n_tiles, grid_y, s);
}

int block_tile_width_fp8(int C, int wclass) { return C == B32_C && wclass != TW_NARROW3 ? Mfma32FP8::TWO : 0; }

}  // namespace conet
