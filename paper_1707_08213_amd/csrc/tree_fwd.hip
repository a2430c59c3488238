// Dispatch of the fused tree forward kernel by window shape, and the write
// probe used to measure the HBM store ceiling.
#include "tree_fwd_kernel.h"

namespace swdft {

int tree_fwd_columns_per_wave(int n0, int n1) {
  (void)n0;
  return 64 / n1;
}

int tree_fwd_rows_per_chunk(int n0, int n1) {
  const int ring = n0 > 1 ? n0 / 2 : 1;
  return n1 > ring ? n1 : ring;
}

hipError_t launch_tree_fwd(int n0, int n1, bool real_input, const void* x, float2* y,
                           const TreeGeom& g, const TwiddlesF32& tw, hipStream_t stream) {
  switch (n0) {
    case 1: return launch_tree_fwd_n0_1(n1, real_input, x, y, g, tw, stream);
    case 2: return launch_tree_fwd_n0_2(n1, real_input, x, y, g, tw, stream);
    case 4: return launch_tree_fwd_n0_4(n1, real_input, x, y, g, tw, stream);
    case 8: return launch_tree_fwd_n0_8(n1, real_input, x, y, g, tw, stream);
    case 16: return launch_tree_fwd_n0_16(n1, real_input, x, y, g, tw, stream);
    case 32: return launch_tree_fwd_n0_32(n1, real_input, x, y, g, tw, stream);
    default: return hipErrorInvalidValue;
  }
}

namespace {
__global__ __launch_bounds__(256) void write_probe_kernel(float2* __restrict__ y, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const float2 v = make_float2(1.0f, -1.0f);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    tree::store_nt(y + i, v);
  }
}
}  // namespace

hipError_t launch_write_probe(float2* y, int64_t n_float2, hipStream_t stream) {
  const int64_t per_block = 256 * 16;
  int64_t blocks = (n_float2 + per_block - 1) / per_block;
  if (blocks < 1) blocks = 1;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(write_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, y, n_float2);
  return hipGetLastError();
}

}  // namespace swdft
