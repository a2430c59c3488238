// Symbols of the persistent class kernels of batched plans and the counter
// reset kernel (see batched.h).
#include "batched.h"

namespace swdft {

const void* batched_tree_symbol_r(int n0, int n1);
const void* batched_tree_symbol_c(int n0, int n1);
const void* batched_dense_symbol_r(int n0, int n1);
const void* batched_dense_symbol_c(int n0, int n1);

namespace {
// Clears `n` work counters; runs first in a batched plan's graph.
__global__ void reset_counters_kernel(unsigned* counters, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) counters[i] = 0u;
}
}  // namespace

bool batched_shape_supported(int n0, int n1) {
  auto ok = [](int n) { return n == 8 || n == 16 || n == 32; };
  return ok(n0) && ok(n1);
}

// Lanes per column stream of the class kernels: the single-plan default, so
// that a batched image and a single plan of it give identical bits.
int batched_tree_kg(int n0, int n1) { return batched_kg(n0, n1); }

const void* batched_tree_symbol(int n0, int n1, bool real_input) {
  return real_input ? batched_tree_symbol_r(n0, n1) : batched_tree_symbol_c(n0, n1);
}

const void* batched_dense_symbol(int n0, int n1, bool real_input) {
  return real_input ? batched_dense_symbol_r(n0, n1) : batched_dense_symbol_c(n0, n1);
}

const void* batched_reset_symbol() { return reinterpret_cast<const void*>(&reset_counters_kernel); }

}  // namespace swdft
