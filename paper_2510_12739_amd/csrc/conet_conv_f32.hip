// F32 instantiations of the 3x3 conv kernels (one translation unit per dtype).
#include "conet_conv_impl.h"

namespace conet {

hipError_t launch_conv_f32(int mode, int cin, int cout, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  return launch_dtype<ArithF32>(mode, cin, cout, a, n_tiles, grid_y, s);
}

int conv_tile_width_f32(int cin, int cout) { return tile_width_dtype<ArithF32>(cin, cout); }
int conv_tile_width_narrow_f32(int cin, int cout) { return tile_width_narrow_dtype<ArithF32>(cin, cout); }

}  // namespace conet
