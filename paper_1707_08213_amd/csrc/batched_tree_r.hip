// Persistent tree class kernels of batched plans, real input (see batched_kernels.h).
#include "batched_kernels.h"

namespace swdft {
const void* batched_tree_symbol_r(int n0, int n1) {
  return batched::class_symbol<true, false>(n0, n1);
}
}  // namespace swdft
