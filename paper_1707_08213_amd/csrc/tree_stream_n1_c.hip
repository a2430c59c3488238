// Streaming 2D tree kernels with n0 = 1, complex input (every n1);
// see tree_stream_kernel.h.
#include "tree_stream_kernel.h"

namespace swdft {
hipError_t launch_tree_stream_n0_1_c(int n1, const void* x, float2* y, float2* state, const StreamGeom& g, const TwiddlesF32& tw, hipStream_t s) {
  return tree::launch_stream_n0<1, false>(n1, x, y, state, g, tw, s);
}
}  // namespace swdft
