// Per-window FFT kernels (the SWFFT comparator), real input; see
// swfft_kernel.h.
#include "swfft_kernel.h"

namespace swdft {
hipError_t launch_swfft_r(int n0, int n1, const void* x, float2* y, const SwfftGeom& g,
                          const TwiddlesF32& tw, hipStream_t s) {
  return swfft::launch<true>(n0, n1, x, y, g, tw, s);
}
}  // namespace swdft
