// Fused tree forward kernels with n0 = 2 (every n1); see tree_fwd_kernel.h.
#include "tree_fwd_kernel.h"

namespace swdft {
hipError_t launch_tree_fwd_n0_2(int n1, bool real_input, const void* x, float2* y,
                                  const TreeGeom& g, const TwiddlesF32& tw, hipStream_t s) {
  return tree::launch_n0<2>(n1, real_input, x, y, g, tw, s);
}
}  // namespace swdft
