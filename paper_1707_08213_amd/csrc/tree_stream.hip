// Dispatch of the streaming 2D tree kernel by window shape, and the fill
// kernel that clears a stream's resident state.
#include "plan.h"
#include "tree_stream_kernel.h"

namespace swdft {

int tree_stream_kg(int n0) { return tree::stream_kg(n0); }

// Ring values per lane of the resident state (a split stream keeps its
// residue's share).
int tree_stream_state_slots(int n0) {
  switch (n0) {
    case 1: return tree::ColCfg<1, tree::stream_kg(1)>::RING_TOTAL;
    case 2: return tree::ColCfg<2, tree::stream_kg(2)>::RING_TOTAL;
    case 4: return tree::ColCfg<4, tree::stream_kg(4)>::RING_TOTAL;
    case 8: return tree::ColCfg<8, tree::stream_kg(8)>::RING_TOTAL;
    case 16: return tree::ColCfg<16, tree::stream_kg(16)>::RING_TOTAL;
    case 32: return tree::ColCfg<32, tree::stream_kg(32)>::RING_TOTAL;
    default: return 0;
  }
}

namespace {
__global__ __launch_bounds__(256) void fill_zero_kernel(float2* __restrict__ p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = make_float2(0.f, 0.f);
}
}  // namespace

hipError_t launch_fill_zero(float2* p, int64_t n, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t launch_tree_stream(int n0, int n1, bool real_input, const void* x, float2* y,
                              float2* state, const StreamGeom& g, const TwiddlesF32& tw,
                              hipStream_t stream) {
  switch (n0) {
    case 1: return real_input ? launch_tree_stream_n0_1_r(n1, x, y, state, g, tw, stream) : launch_tree_stream_n0_1_c(n1, x, y, state, g, tw, stream);
    case 2: return real_input ? launch_tree_stream_n0_2_r(n1, x, y, state, g, tw, stream) : launch_tree_stream_n0_2_c(n1, x, y, state, g, tw, stream);
    case 4: return real_input ? launch_tree_stream_n0_4_r(n1, x, y, state, g, tw, stream) : launch_tree_stream_n0_4_c(n1, x, y, state, g, tw, stream);
    case 8: return real_input ? launch_tree_stream_n0_8_r(n1, x, y, state, g, tw, stream) : launch_tree_stream_n0_8_c(n1, x, y, state, g, tw, stream);
    case 16: return real_input ? launch_tree_stream_n0_16_r(n1, x, y, state, g, tw, stream) : launch_tree_stream_n0_16_c(n1, x, y, state, g, tw, stream);
    case 32: return real_input ? launch_tree_stream_n0_32_r(n1, x, y, state, g, tw, stream) : launch_tree_stream_n0_32_c(n1, x, y, state, g, tw, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace swdft
