// Dispatch of the adjoint tree kernels by window shape.
#include "tree_adj_kernel.h"

namespace swdft {

int tree_adj_rows_per_chunk(int n0, int n1, int kg) {
  const int ring = n0 > 1 ? n0 / 2 : 1;
  const int pf = tree::adj_prefetch_rows(n0);
  const int r = n1 * kg;
  int cr = r > ring ? r : ring;
  return cr > pf ? cr : pf;
}

static_assert(tree::AdjCfg<16, 16, 1>::CR == 16 && tree::AdjCfg<2, 1, 1>::CR == 4 &&
                  tree::AdjCfg<32, 8, 1>::CR == 16 && tree::AdjCfg<4, 2, 1>::CR == 4 &&
                  tree::AdjCfg<32, 8, 2>::CR == 16 && tree::AdjCfg<16, 16, 2>::CR == 32,
              "host and kernel rows per chunk agree");

int tree_adj_columns_per_wave(int n0, int n1, int kg) {
  (void)n0;
  return 64 / (n1 * kg);
}

// n0 = 32 splits its streams over two lanes: the unsplit rings and two
// prefetched rows needed 256 VGPRs, 256 AGPRs and scratch.
int tree_adj_default_kg(int n0, int n1) { return n0 == 32 && n1 <= 32 ? 2 : 1; }

bool tree_adj_kg_supported(int n0, int n1, int kg) { return tree::adj_kg_built(n0, n1, kg); }

int64_t tree_adj_workspace_elems(int n0, int n1, const AdjGeom& g) {
  (void)n0;
  const int64_t wcols = 64 / (n1 * g.kg) + n1 - 1;
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
