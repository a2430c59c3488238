// Dispatch of the 3D adjoint tree kernels by window shape.
#include "tree3d_adj_kernel.h"

namespace swdft {

int tree3_adj_rows_per_chunk(int n0, int n1, int n2) {
  const int ring = n0 > 1 ? n0 / 2 : 1;
  const int pf = n0 <= 8 ? 4 : 2;
  int cr = n1 > n2 ? n1 : n2;
  cr = cr > ring ? cr : ring;
  return cr > pf ? cr : pf;
}

static_assert(tree3::Adj3Cfg<8, 8, 8>::CR == 8 && tree3::Adj3Cfg<2, 2, 2>::CR == 4 &&
                  tree3::Adj3Cfg<16, 2, 4>::CR == 8,
              "host and kernel rows per chunk agree");

int64_t tree3_adj_workspace_elems(int n1, int n2, const Adj3Geom& g) {
  const int64_t qw = 64 / (n1 * n2);
  return (int64_t)g.batch * g.P1 * g.nstrips * g.N0 * n1 * (qw + n2 - 1);
}

hipError_t launch_tree3_adj(int n0, int n1, int n2, bool real_input, const float2* dy, void* ws,
                            void* dx, const Adj3Geom& g, const Twiddles3F32& tw,
                            hipStream_t stream) {
  switch (n0) {
    case 2: return real_input ? launch_tree3_adj_n0_2_r(n1, n2, dy, ws, dx, g, tw, stream) : launch_tree3_adj_n0_2_c(n1, n2, dy, ws, dx, g, tw, stream);
    case 4: return real_input ? launch_tree3_adj_n0_4_r(n1, n2, dy, ws, dx, g, tw, stream) : launch_tree3_adj_n0_4_c(n1, n2, dy, ws, dx, g, tw, stream);
    case 8: return real_input ? launch_tree3_adj_n0_8_r(n1, n2, dy, ws, dx, g, tw, stream) : launch_tree3_adj_n0_8_c(n1, n2, dy, ws, dx, g, tw, stream);
    case 16: return real_input ? launch_tree3_adj_n0_16_r(n1, n2, dy, ws, dx, g, tw, stream) : launch_tree3_adj_n0_16_c(n1, n2, dy, ws, dx, g, tw, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace swdft
