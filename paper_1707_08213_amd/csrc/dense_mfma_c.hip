// Dense matrix-core kernels for complex input; see dense_mfma_kernel.h.
#include "dense_mfma_kernel.h"

namespace swdft {
hipError_t launch_dense_fwd_c(int n0, int n1, const void* x, float2* y, const DenseGeom& g,
                              const TwiddlesF32& tw, hipStream_t s) {
  return dense::launch<false>(n0, n1, x, y, g, tw, s);
}
}  // namespace swdft
