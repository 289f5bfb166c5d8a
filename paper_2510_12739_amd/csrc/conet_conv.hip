// Dtype dispatch of the 3x3 conv kernels (kernel bodies: conet_conv_impl.h) and of the
// fused block kernel (conet_block_impl.h).
#include "conet_kernels.h"

namespace conet {

hipError_t launch_conv_f32(int mode, int cin, int cout, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s);
hipError_t launch_conv_bf16(int mode, int cin, int cout, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s);
hipError_t launch_conv_fp8(int mode, int cin, int cout, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s);
int conv_tile_width_f32(int cin, int cout);
int conv_tile_width_bf16(int cin, int cout);
int conv_tile_width_fp8(int cin, int cout);
int conv_tile_width_narrow_f32(int cin, int cout);
int conv_tile_width_narrow_bf16(int cin, int cout);
int conv_tile_width_narrow_fp8(int cin, int cout);
hipError_t launch_block_bf16(int kind, int wclass, int C, BlockArgs& a, int n_tiles, int grid_y, hipStream_t s);
int block_tile_width_bf16(int C, int wclass);
hipError_t launch_block_fp8(int kind, int wclass, int C, BlockArgs& a, int n_tiles, int grid_y, hipStream_t s);
int block_tile_width_fp8(int C, int wclass);

hipError_t launch_conv(int dtype, int mode, int cin, int cout, ConvArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  switch (dtype) {
    case DT_F32: return launch_conv_f32(mode, cin, cout, a, n_tiles, grid_y, s);
    case DT_BF16: return launch_conv_bf16(mode, cin, cout, a, n_tiles, grid_y, s);
    case DT_FP8: return launch_conv_fp8(mode, cin, cout, a, n_tiles, grid_y, s);
  }
  return hipErrorInvalidValue;
}

int conv_tile_width(int dtype, int cin, int cout) {
  switch (dtype) {
    case DT_F32: return conv_tile_width_f32(cin, cout);
    case DT_BF16: return conv_tile_width_bf16(cin, cout);
    case DT_FP8: return conv_tile_width_fp8(cin, cout);
  }
  return 0;
}

int conv_tile_width_narrow(int dtype, int cin, int cout) {
  switch (dtype) {
    case DT_F32: return conv_tile_width_narrow_f32(cin, cout);
    case DT_BF16: return conv_tile_width_narrow_bf16(cin, cout);
    case DT_FP8: return conv_tile_width_narrow_fp8(cin, cout);
  }
  return 0;
}

bool conv_supported(int dtype, int cin, int cout) { return conv_tile_width(dtype, cin, cout) > 0; }

int block_tile_width(int dtype, int C, int K, int wclass, bool train) {
  if (K < 1 || K > BLOCK_KMAX) return 0;
  if (train && block_uses_mfma32(dtype, C)) return 0;
  switch (dtype) {
    case DT_BF16: return block_tile_width_bf16(C, wclass);
    case DT_FP8: return block_tile_width_fp8(C, wclass);
  }
  return 0;
}

hipError_t launch_block(int dtype, int kind, int wclass, int C, BlockArgs& a, int n_tiles, int grid_y, hipStream_t s) {
  switch (dtype) {
    case DT_BF16: return launch_block_bf16(kind, wclass, C, a, n_tiles, grid_y, s);
    case DT_FP8: return launch_block_fp8(kind, wclass, C, a, n_tiles, grid_y, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace conet
