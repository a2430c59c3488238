// Dispatch of the fused tree forward kernel by window shape.
#include "tree_fwd_kernel.h"

namespace swdft {

int tree_fwd_columns_per_wave(int n0, int n1, int kg) {
  (void)n0;
  return 64 / (n1 * kg);
}

int tree_fwd_rows_per_chunk(int n0, int n1, int kg, int wv) {
  const int ring = n0 > 1 ? n0 / 2 : 1;
  const int rows_per_pass = n1 * kg * wv;
  return rows_per_pass > ring ? rows_per_pass : ring;
}

// A stream is split over two lanes for n0 = 8, whose short output rows per
// wave need more waves in flight; for n1 = 8, where the two lanes of a stream
// write adjacent 64-byte k0 rows, so each store instruction covers whole
// 128-byte lines; for n0 = 32 with n1 <= 8; and for 16 x 4 (1024^2: 127 ->
// 104 us). n0 = 32 with n1 >= 16 keeps whole streams on whole columns (32 x 16:
// 783 -> 637 us). n0 = 64 is built with one split per n1 (tree::tree_kg64).
int tree_fwd_default_kg(int n0, int n1) {
  if (n0 == 64) return tree::tree_kg64(n1);
  if (n0 == 32) return n1 <= 8 ? 2 : 1;
  if (n0 == 16 && n1 == 4) return 2;
  return (n0 == 8 && n1 <= 32) || (n0 >= 8 && n1 == 8) ? 2 : 1;
}

int tree_fwd_resident_waves(int wpc, int ncu) { return wpc > 0 && ncu > 0 ? wpc * ncu : 0; }

bool tree_fwd_wv_supported(int n0, int kg, int wv) { return tree::tree_wv_built(n0, kg, wv); }

bool tree_fwd_kg_supported(int n0, int n1, int kg) { return tree::tree_kg_built(n0, n1, kg); }

hipError_t launch_tree_fwd(int n0, int n1, bool real_input, const void* x, float2* y,
                           const TreeGeom& g, const TwiddlesF32& tw, hipStream_t stream) {
  switch (n0) {
    case 1: return real_input ? launch_tree_fwd_n0_1_r(n1, x, y, g, tw, stream) : launch_tree_fwd_n0_1_c(n1, x, y, g, tw, stream);
    case 2: return real_input ? launch_tree_fwd_n0_2_r(n1, x, y, g, tw, stream) : launch_tree_fwd_n0_2_c(n1, x, y, g, tw, stream);
    case 4: return real_input ? launch_tree_fwd_n0_4_r(n1, x, y, g, tw, stream) : launch_tree_fwd_n0_4_c(n1, x, y, g, tw, stream);
    case 8: return real_input ? launch_tree_fwd_n0_8_r(n1, x, y, g, tw, stream) : launch_tree_fwd_n0_8_c(n1, x, y, g, tw, stream);
    case 16: return real_input ? launch_tree_fwd_n0_16_r(n1, x, y, g, tw, stream) : launch_tree_fwd_n0_16_c(n1, x, y, g, tw, stream);
    case 32: return real_input ? launch_tree_fwd_n0_32_r(n1, x, y, g, tw, stream) : launch_tree_fwd_n0_32_c(n1, x, y, g, tw, stream);
    case 64: return real_input ? launch_tree_fwd_n0_64_r(n1, x, y, g, tw, stream) : launch_tree_fwd_n0_64_c(n1, x, y, g, tw, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace swdft
