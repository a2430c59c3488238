// Adjoint tree kernels with n0 = 2, real input (every n1);
// see tree_adj_kernel.h.
#include "tree_adj_kernel.h"

namespace swdft {
hipError_t launch_tree_adj_n0_2_r(int n1, const float2* dy, void* ws, void* dx, const AdjGeom& g, const TwiddlesF32& tw, hipStream_t s) {
  return tree::launch_adj_n0<2, true>(n1, dy, ws, dx, g, tw, s);
}
}  // namespace swdft
