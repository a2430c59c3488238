// Persistent dense class kernels of batched plans, complex input (see batched_kernels.h).
#include "batched_kernels.h"

namespace swdft {
const void* batched_dense_symbol_c(int n0, int n1) {
  return batched::class_symbol<false, true>(n0, n1);
}
}  // namespace swdft
