// 3D adjoint tree kernels with n0 = 4, complex input (every n1, n2);
// see tree3d_adj_kernel.h.
#include "tree3d_adj_kernel.h"

namespace swdft {
hipError_t launch_tree3_adj_n0_4_c(int n1, int n2, const float2* dy, void* ws, void* dx, const Adj3Geom& g, const Twiddles3F32& tw, hipStream_t s) {
  return tree3::launch3_adj_n0<4, false>(n1, n2, dy, ws, dx, g, tw, s);
}
}  // namespace swdft
