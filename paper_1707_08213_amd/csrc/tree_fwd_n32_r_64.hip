// Forward tree kernels with n0 = 32, n1 = 64, real input; see
// tree_fwd_kernel.h.
#include "tree_fwd_kernel.h"

namespace swdft {
namespace tree {
template hipError_t launch_one<32, 64, true>(const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
}  // namespace tree
}  // namespace swdft
