// Mixed-radix forward tree kernels with a power-of-two n0 (4, 8, 16) and
// n1 in {3, 6, 9, 12, 24}, real input; see tree_mixed_kernel.h.
#include "tree_mixed_kernel.h"

namespace swdft {
hipError_t launch_tree_mixed_n0_4_r(int n1, const void* x, float2* y, const TreeGeom& g,
                                     const TwiddlesF32& tw, hipStream_t s) {
  return mixed::launch_n0<4, true>(n1, x, y, g, tw, s);
}
hipError_t launch_tree_mixed_n0_8_r(int n1, const void* x, float2* y, const TreeGeom& g,
                                     const TwiddlesF32& tw, hipStream_t s) {
  return mixed::launch_n0<8, true>(n1, x, y, g, tw, s);
}
hipError_t launch_tree_mixed_n0_16_r(int n1, const void* x, float2* y, const TreeGeom& g,
                                     const TwiddlesF32& tw, hipStream_t s) {
  return mixed::launch_n0<16, true>(n1, x, y, g, tw, s);
}
}  // namespace swdft
