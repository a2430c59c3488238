// Two-wave forward tree kernels whose first chunk holds only priming steps
// (n1 = 1, n0 = 8, 16, 32), compiled to assembly by test_lds_order.py to check
// that every LDS read of a chunk's column phase precedes the barrier that
// lets the other wave write the next chunk's rows.
#include "tree_fwd_kernel.h"

namespace swdft {
namespace tree {
template hipError_t launch_cfg<8, 1, true, 2, 2>(const void*, float2*, const TreeGeom&,
                                                 const TwiddlesF32&, hipStream_t);
template hipError_t launch_cfg<16, 1, true, 1, 2>(const void*, float2*, const TreeGeom&,
                                                  const TwiddlesF32&, hipStream_t);
template hipError_t launch_cfg<32, 1, true, 2, 2>(const void*, float2*, const TreeGeom&,
                                                  const TwiddlesF32&, hipStream_t);
}  // namespace tree
}  // namespace swdft
