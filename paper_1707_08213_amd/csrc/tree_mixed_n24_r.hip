// Mixed-radix forward tree kernels with n0 = 24, real input (every
// n1); see tree_mixed_kernel.h.
#include "tree_mixed_kernel.h"

namespace swdft {
hipError_t launch_tree_mixed_n0_24_r(int n1, const void* x, float2* y, const TreeGeom& g,
                                     const TwiddlesF32& tw, hipStream_t s) {
  return mixed::launch_n0<24, true>(n1, x, y, g, tw, s);
}
}  // namespace swdft
