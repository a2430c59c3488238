// Forward tree kernels with n0 = 16, real input (every n1; n1 = 16, 32
// and 64 are instantiated in tree_fwd_n16_r_16.hip, _32.hip and _64.hip so that the
// largest kernels compile in parallel); see tree_fwd_kernel.h.
#include "tree_fwd_kernel.h"

namespace swdft {
namespace tree {
extern template hipError_t launch_one<16, 16, true>(const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
extern template hipError_t launch_one<16, 32, true>(const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
extern template hipError_t launch_one<16, 64, true>(const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
}  // namespace tree

hipError_t launch_tree_fwd_n0_16_r(int n1, const void* x, float2* y, const TreeGeom& g, const TwiddlesF32& tw, hipStream_t s) {
  return tree::launch_n0<16, true>(n1, x, y, g, tw, s);
}
}  // namespace swdft
