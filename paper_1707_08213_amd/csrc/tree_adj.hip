// Dispatch of the adjoint tree kernels by window shape.
#include "tree_adj_kernel.h"

namespace swdft {

int tree_adj_rows_per_chunk(int n0, int n1) {
  const int ring = n0 > 1 ? n0 / 2 : 1;
  const int pf = tree::adj_prefetch_rows(n0);
  int cr = n1 > ring ? n1 : ring;
  return cr > pf ? cr : pf;
}

static_assert(tree::AdjCfg<16, 16>::CR == 16 && tree::AdjCfg<2, 1>::CR == 4 &&
                  tree::AdjCfg<32, 8>::CR == 16 && tree::AdjCfg<4, 2>::CR == 4,
              "host and kernel rows per chunk agree");

int tree_adj_columns_per_wave(int n0, int n1) {
  (void)n0;
  return 64 / n1;
}

int64_t tree_adj_workspace_elems(int n0, int n1, const AdjGeom& g) {
  (void)n0;
  const int64_t wcols = 64 / n1 + n1 - 1;
  return (int64_t)g.batch * g.nstrips * g.N0 * wcols;
}

hipError_t launch_tree_adj(int n0, int n1, bool real_input, const float2* dy, void* ws, void* dx,
                           const AdjGeom& g, const TwiddlesF32& tw, hipStream_t stream) {
  switch (n0) {
    case 1: return real_input ? launch_tree_adj_n0_1_r(n1, dy, ws, dx, g, tw, stream) : launch_tree_adj_n0_1_c(n1, dy, ws, dx, g, tw, stream);
    case 2: return real_input ? launch_tree_adj_n0_2_r(n1, dy, ws, dx, g, tw, stream) : launch_tree_adj_n0_2_c(n1, dy, ws, dx, g, tw, stream);
    case 4: return real_input ? launch_tree_adj_n0_4_r(n1, dy, ws, dx, g, tw, stream) : launch_tree_adj_n0_4_c(n1, dy, ws, dx, g, tw, stream);
    case 8: return real_input ? launch_tree_adj_n0_8_r(n1, dy, ws, dx, g, tw, stream) : launch_tree_adj_n0_8_c(n1, dy, ws, dx, g, tw, stream);
    case 16: return real_input ? launch_tree_adj_n0_16_r(n1, dy, ws, dx, g, tw, stream) : launch_tree_adj_n0_16_c(n1, dy, ws, dx, g, tw, stream);
    case 32: return real_input ? launch_tree_adj_n0_32_r(n1, dy, ws, dx, g, tw, stream) : launch_tree_adj_n0_32_c(n1, dy, ws, dx, g, tw, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace swdft
