// Forward tree kernels with n0 = 16, real input (every n1);
// see tree_fwd_kernel.h.
#include "tree_fwd_kernel.h"

namespace swdft {
hipError_t launch_tree_fwd_n0_16_r(int n1, const void* x, float2* y, const TreeGeom& g, const TwiddlesF32& tw, hipStream_t s) {
  return tree::launch_n0<16, true>(n1, x, y, g, tw, s);
}
}  // namespace swdft
