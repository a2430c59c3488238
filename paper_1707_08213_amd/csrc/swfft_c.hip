// Per-window FFT kernels (the SWFFT comparator), complex input; see
// swfft_kernel.h.
#include "swfft_kernel.h"

namespace swdft {
hipError_t launch_swfft_c(int n0, int n1, const void* x, float2* y, const SwfftGeom& g,
                          const TwiddlesF32& tw, hipStream_t s) {
  return swfft::launch<false>(n0, n1, x, y, g, tw, s);
}

int swfft_windows_per_group(int n0, int n1) { return 64 / (n0 > n1 ? n0 : n1); }

hipError_t launch_swfft(int n0, int n1, bool real_input, const void* x, float2* y,
                        const SwfftGeom& g, const TwiddlesF32& tw, hipStream_t stream) {
  return real_input ? launch_swfft_r(n0, n1, x, y, g, tw, stream)
                    : launch_swfft_c(n0, n1, x, y, g, tw, stream);
}
}  // namespace swdft
