// Dispatch of the dense matrix-core kernels (see dense_mfma_kernel.h).
#include "internal.h"

namespace swdft {

hipError_t launch_dense_fwd_r(int, int, const void*, float2*, const DenseGeom&, const TwiddlesF32&,
                              hipStream_t);
hipError_t launch_dense_fwd_c(int, int, const void*, float2*, const DenseGeom&, const TwiddlesF32&,
                              hipStream_t);

bool dense_supported(int n0, int n1) {
  auto ok = [](int n) { return n == 8 || n == 16 || n == 32; };
  return ok(n0) && ok(n1);
}

int dense_columns_per_wave(int n0, int n1) {
  (void)n0;
  return n1 >= 16 ? 1 : 16 / n1;
}

hipError_t launch_dense_fwd(int n0, int n1, bool real_input, const void* x, float2* y,
                            const DenseGeom& g, const TwiddlesF32& tw, hipStream_t stream) {
  return real_input ? launch_dense_fwd_r(n0, n1, x, y, g, tw, stream)
                    : launch_dense_fwd_c(n0, n1, x, y, g, tw, stream);
}

}  // namespace swdft
