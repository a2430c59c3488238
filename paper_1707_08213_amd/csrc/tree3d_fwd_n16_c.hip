// 3D forward tree kernels with n0 = 16, complex input (every n1, n2);
// see tree3d_fwd_kernel.h.
#include "tree3d_fwd_kernel.h"

namespace swdft {
hipError_t launch_tree3_fwd_n0_16_c(int n1, int n2, const void* x, float2* y, const Tree3Geom& g, const Twiddles3F32& tw, hipStream_t s) {
  return tree3::launch3_n0<16, false>(n1, n2, x, y, g, tw, s);
}
}  // namespace swdft
