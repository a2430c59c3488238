// Forward tree kernels with n0 = 64, n1 = 16, complex input; see
// tree_fwd_kernel.h.
#include "tree_fwd_kernel.h"

namespace swdft {
namespace tree {
template hipError_t launch_one<64, 16, false>(const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
}  // namespace tree
}  // namespace swdft
