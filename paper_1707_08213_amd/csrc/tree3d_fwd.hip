// Dispatch of the fused 3D tree forward kernel by window shape.
#include "tree3d_fwd_kernel.h"

namespace swdft {

bool tree3_shape_supported(int n0, int n1, int n2) {
  auto side = [](int n) { return n == 2 || n == 4 || n == 8; };
  return (side(n0) || n0 == 16) && side(n1) && side(n2);
}

int tree3_columns_per_wave(int n1, int n2) { return 64 / (n1 * n2); }

int tree3_rows_per_chunk(int n0, int n1, int n2) {
  const int ring = n0 > 1 ? n0 / 2 : 1;
  const int r = n1 > n2 ? n1 : n2;
  return r > ring ? r : ring;
}

hipError_t launch_tree3_fwd(int n0, int n1, int n2, bool real_input, const void* x, float2* y,
                            const Tree3Geom& g, const Twiddles3F32& tw, hipStream_t stream) {
  switch (n0) {
    case 2: return real_input ? launch_tree3_fwd_n0_2_r(n1, n2, x, y, g, tw, stream) : launch_tree3_fwd_n0_2_c(n1, n2, x, y, g, tw, stream);
    case 4: return real_input ? launch_tree3_fwd_n0_4_r(n1, n2, x, y, g, tw, stream) : launch_tree3_fwd_n0_4_c(n1, n2, x, y, g, tw, stream);
    case 8: return real_input ? launch_tree3_fwd_n0_8_r(n1, n2, x, y, g, tw, stream) : launch_tree3_fwd_n0_8_c(n1, n2, x, y, g, tw, stream);
    case 16: return real_input ? launch_tree3_fwd_n0_16_r(n1, n2, x, y, g, tw, stream) : launch_tree3_fwd_n0_16_c(n1, n2, x, y, g, tw, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace swdft
