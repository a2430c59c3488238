// Dispatch of the adjoint tree kernels by window shape.
#include "tree_adj_kernel.h"

namespace swdft {

int tree_adj_rows_per_chunk(int n0, int n1) {
  const int ring = n0 > 1 ? n0 / 2 : 1;
  int cr = n1 > ring ? n1 : ring;
  return cr > 2 ? cr : 2;
}

int64_t tree_adj_workspace_elems(int n0, int n1, const AdjGeom& g) {
  (void)n0;
  const int64_t wcols = 64 / n1 + n1 - 1;
  return (int64_t)g.batch * g.nstrips * g.N0 * wcols;
}

hipError_t launch_tree_adj(int n0, int n1, bool real_input, const float2* dy, void* ws, void* dx,
                           const AdjGeom& g, const TwiddlesF32& tw, hipStream_t stream) {
  switch (n0) {
    case 1: return launch_tree_adj_n0_1(n1, real_input, dy, ws, dx, g, tw, stream);
    case 2: return launch_tree_adj_n0_2(n1, real_input, dy, ws, dx, g, tw, stream);
    case 4: return launch_tree_adj_n0_4(n1, real_input, dy, ws, dx, g, tw, stream);
    case 8: return launch_tree_adj_n0_8(n1, real_input, dy, ws, dx, g, tw, stream);
    case 16: return launch_tree_adj_n0_16(n1, real_input, dy, ws, dx, g, tw, stream);
    case 32: return launch_tree_adj_n0_32(n1, real_input, dy, ws, dx, g, tw, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace swdft
