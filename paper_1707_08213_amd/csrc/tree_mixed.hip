// Dispatch and launch shape of the mixed-radix tree kernels by window shape;
// see tree_mixed_kernel.h.
#include "tree_mixed_kernel.h"

namespace swdft {

hipError_t launch_tree_mixed_n0_3_r(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_3_c(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_4_r(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_4_c(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_6_r(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_6_c(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_8_r(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_8_c(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_9_r(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_9_c(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_12_r(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_12_c(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_16_r(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_16_c(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_24_r(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);
hipError_t launch_tree_mixed_n0_24_c(int, const void*, float2*, const TreeGeom&, const TwiddlesF32&, hipStream_t);

namespace {

constexpr bool pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
constexpr bool side_built(int n) {
  return n == 3 || n == 4 || n == 6 || n == 8 || n == 9 || n == 12 || n == 16 || n == 24;
}

}  // namespace

bool tree_mixed_supported(int n0, int n1) {
  return side_built(n0) && side_built(n1) && !(pow2(n0) && pow2(n1));
}

int tree_mixed_rows_per_chunk(int n0, int n1) { return mixed::rows_per_chunk(n0, n1); }

hipError_t launch_tree_mixed_r(int n0, int n1, const void* x, float2* y, const TreeGeom& g,
                               const TwiddlesF32& tw, hipStream_t s) {
  switch (n0) {
    case 3: return launch_tree_mixed_n0_3_r(n1, x, y, g, tw, s);
    case 4: return launch_tree_mixed_n0_4_r(n1, x, y, g, tw, s);
    case 6: return launch_tree_mixed_n0_6_r(n1, x, y, g, tw, s);
    case 8: return launch_tree_mixed_n0_8_r(n1, x, y, g, tw, s);
    case 9: return launch_tree_mixed_n0_9_r(n1, x, y, g, tw, s);
    case 12: return launch_tree_mixed_n0_12_r(n1, x, y, g, tw, s);
    case 16: return launch_tree_mixed_n0_16_r(n1, x, y, g, tw, s);
    case 24: return launch_tree_mixed_n0_24_r(n1, x, y, g, tw, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tree_mixed_c(int n0, int n1, const void* x, float2* y, const TreeGeom& g,
                               const TwiddlesF32& tw, hipStream_t s) {
  switch (n0) {
    case 3: return launch_tree_mixed_n0_3_c(n1, x, y, g, tw, s);
    case 4: return launch_tree_mixed_n0_4_c(n1, x, y, g, tw, s);
    case 6: return launch_tree_mixed_n0_6_c(n1, x, y, g, tw, s);
    case 8: return launch_tree_mixed_n0_8_c(n1, x, y, g, tw, s);
    case 9: return launch_tree_mixed_n0_9_c(n1, x, y, g, tw, s);
    case 12: return launch_tree_mixed_n0_12_c(n1, x, y, g, tw, s);
    case 16: return launch_tree_mixed_n0_16_c(n1, x, y, g, tw, s);
    case 24: return launch_tree_mixed_n0_24_c(n1, x, y, g, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace swdft
