// Fused forward 3D Tree SWDFT for gfx950 (the k-dimensional extension of
// Sec. 4.4, k = 3).
//
// The trees of the 3D extension run m2 levels along axis 2, then m1 along
// axis 1, then m0 along axis 0 (the three level equations that instantiate
// Eq. (7)); the last level is the 3D DFT of every window. Along axis 0 the
// trees share nodes between window rows exactly as in 2D, so the kernel
// keeps the 2D design there (register rings streamed down a slab of window
// rows) and computes the levels of axes 2 and 1 per window position, as the
// 2D kernel does for its row levels:
//  * Plane phase, per chunk of CR input planes p0 and the strip's QW windows
//    at (q1, q2_0 + c):
//      pass A: lane (r, c, j1) runs the m2 levels of axis 2 on the n2 inputs
//        x[p0][q1 + j1][q2 + 0..n2-1] (Eq. (5) along the last axis) and
//        leaves the n2 bins in LDS;
//      pass B: lane (r, c, k2) runs the m1 levels of axis 1 on the n1 values
//        of its column and writes the n1 bins back in place.
//    LDS then holds Z[p0][c][k1][k2], the (n1 x n2) DFT of the plane patch.
//  * Column phase: lane (c, k1, k2) owns the stream Z[.][c][k1][k2] and walks
//    down the slab through the m0 levels of axis 0 (Eq. (6) with the node
//    index ranging over (k1, k2) pairs), storing the last level at once.
//  * Output y[b][q0][q1][q2][k0][k1][k2]: for each k0 the 64 lanes store QW
//    runs of n1*n2 complex values through a buffer resource per output row
//    (empty for priming rows, and ending at the last window of the strip);
//    non-temporal stores when a run is whole 128-byte lines (n1*n2 >= 16),
//    plain stores below that.
//  * Inputs of the next chunk are loaded before the column phase of the
//    current one (the loop is rotated as in the 2D kernel), from clamped
//    in-range addresses, with zeros selected past the volume's edges.
// Window sides: n0 in {2, 4, 8, 16}, n1 and n2 in {2, 4, 8}.
#pragma once

#include "tree_fwd_kernel.h"

namespace swdft {
namespace tree3 {

using tree::buf_rsrc;
using tree::column_levels;
using tree::ColCfg;
using tree::row_levels;
using tree::sfor;
using tree::store_buf;
using tree::uniform_copy;
using tree::uload;

template <int N0W, int N1W, int N2W, bool REAL>
struct Tree3Cfg {
  static constexpr int NK = N1W * N2W;       // (k1, k2) pairs of a window
  static constexpr int QW = 64 / NK;         // windows per strip (along axis 2)
  // non-temporal stores only where one store instruction writes whole
  // 128-byte lines of a window (NK complex64 values per k0 row, NK >= 16);
  // narrower rows take plain stores, which L2 merges (128^3 / 16x2x2:
  // 817 us with non-temporal partial lines)
  static constexpr bool NT_STORES = NK >= 16;
  static constexpr int RING = N0W > 1 ? N0W / 2 : 1;
  static constexpr int RA = N2W;             // plane rows per pass A (QW*N1W lanes per row)
  static constexpr int RB = N1W;             // plane rows per pass B (QW*N2W lanes per row)
  static constexpr int CR0 = RA > RB ? RA : RB;
  static constexpr int CR = CR0 > RING ? CR0 : RING;  // plane rows per chunk
  static constexpr int PA = CR / RA;         // passes A per chunk
  static constexpr int PB = CR / RB;         // passes B per chunk
  static constexpr int ZS = N2W + 1;         // padded stride of one (c, j1) line in LDS
  static constexpr int ZROW = QW * N1W * ZS; // float2 per plane row in LDS
  static constexpr int LDS_FLOAT2 = CR * ZROW;
  static_assert(NK <= 64 && 64 % NK == 0, "one wave must hold the (k1, k2) plane of a window");
  static_assert(CR % RING == 0, "chunks must start on ring periods");
};

// One tile: window columns [strip*QW, +QW) along axis 2 at window row q1 of
// axis 1, window rows [slab*S, +S) along axis 0, of volume b.
template <int N0W, int N1W, int N2W, bool REAL>
__device__ __forceinline__ void tree3_fwd_tile(const void* __restrict__ xv, float2* __restrict__ y,
                                               const Tree3Geom& g_in, const Twiddles3F32& tw,
                                               int strip, int q1, int slab, int b,
                                               float2* __restrict__ zl) {
  using C = Tree3Cfg<N0W, N1W, N2W, REAL>;
  using CC = ColCfg<N0W, 1>;
  const int lane = threadIdx.x;
  const Tree3Geom g = uniform_copy(g_in);

  const int64_t q2_0 = (int64_t)strip * C::QW;
  const int64_t row0 = (int64_t)slab * g.S;
  const int64_t q0_end = min(row0 + (int64_t)g.S, g.P0);
  const int nrows = (int)(q0_end - row0) + N0W - 1;
  const int nchunks = (nrows + C::CR - 1) / C::CR;

  using XT = std::conditional_t<REAL, float, float2>;
  const XT* ximg = reinterpret_cast<const XT*>(xv) + b * g.x_image_stride;
  float2* yimg = y + b * g.y_image_stride;
  const int64_t plane = g.N1 * g.N2;

  // pass A roles: lane (ra, c, j1)
  const int pa_j1 = lane % N1W;
  const int pa_c = (lane / N1W) % C::QW;
  const int pa_r = lane / (N1W * C::QW);
  // element offset of x[p0 = 0][q1 + j1][q2_0 + c + n2 - 1 - d] within the
  // volume, and whether that column exists
  int64_t a_off[N2W];
  bool a_ok[N2W];
  sfor<0, N2W>([&](auto D) {
    constexpr int d = D;
    const int64_t col = q2_0 + pa_c + (N2W - 1 - d);
    a_ok[d] = col < g.N2;
    a_off[d] = ((int64_t)q1 + pa_j1) * g.N2 + (a_ok[d] ? col : 0);
  });
  // inputs of this lane's passes of one chunk (planes crow + pa * RA + ra),
  // loaded a chunk ahead; planes past the volume read zero
  XT xin[C::PA][N2W];
  auto load_chunk = [&](int64_t crow) __attribute__((always_inline)) {
    sfor<0, C::PA>([&](auto P) {
      constexpr int pa = P;
      const int64_t p0 = crow + pa * C::RA + pa_r;
      const bool row_ok = p0 < g.N0;
      const int64_t base = (row_ok ? p0 : 0) * plane;
      sfor<0, N2W>([&](auto D) {
        constexpr int d = D;
        const XT v = ximg[base + a_off[d]];
        if constexpr (REAL) {
          xin[pa][d] = (row_ok && a_ok[d]) ? v : 0.f;
        } else {
          xin[pa][d] = (row_ok && a_ok[d]) ? v : make_float2(0.f, 0.f);
        }
      });
    });
  };

  // pass B roles: lane (rb, c, k2)
  const int pb_k2 = lane % N2W;
  const int pb_c = (lane / N2W) % C::QW;
  const int pb_r = lane / (N2W * C::QW);

  // column-phase roles: lane (c, k1, k2)
  const int cp_c = lane / C::NK;
  const int cp_k = lane % C::NK;  // k1 * n2 + k2
  const int cp_k1 = cp_k / N2W;
  const int cp_k2 = cp_k % N2W;
  // output of one window row: the strip's QW windows of n0*n1*n2 values
  float2* ystrip = yimg + ((int64_t)q1 * g.P2 + q2_0) * (N0W * C::NK);
  const uint64_t row_bytes = (uint64_t)g.P1 * g.P2 * (N0W * C::NK * sizeof(float2));
  const uint32_t strip_bytes = tree::uniform_u32(
      (uint32_t)(min((int64_t)C::QW, g.P2 - q2_0) * (N0W * C::NK * (int)sizeof(float2))));
  const uint32_t lane_off = (uint32_t)((cp_c * (N0W * C::NK) + cp_k) * (int)sizeof(float2));

  float2 lanefac[CC::M0 + 1];
  float2 lw[CC::M0 + 1][CC::LW];
  sfor<0, CC::M0 + 1>([&](auto U) { lanefac[U] = make_float2(1.f, 0.f); });

  float2 ring[CC::RING_TOTAL];
  sfor<0, CC::RING_TOTAL>([&](auto K) { ring[K] = make_float2(0.f, 0.f); });

  auto plane_phase = [&]() {
    // pass A: axis-2 levels, n2 bins per (plane row, window, j1) line
    sfor<0, C::PA>([&](auto P) {
      constexpr int pa = P;
      float2 v[N2W];
      sfor<0, N2W>([&](auto D) {
        if constexpr (REAL) {
          v[D] = make_float2(xin[pa][D], 0.f);
        } else {
          v[D] = xin[pa][D];
        }
      });
      row_levels<N2W>(v, tw.w2);
      float2* line = zl + (pa * C::RA + pa_r) * C::ZROW + (pa_c * N1W + pa_j1) * C::ZS;
      sfor<0, N2W>([&](auto K) { line[K] = v[K]; });
    });
    __syncthreads();
    // pass B: axis-1 levels over the n1 lines of a window, in place
    sfor<0, C::PB>([&](auto P) {
      constexpr int pb = P;
      float2* col = zl + (pb * C::RB + pb_r) * C::ZROW + pb_c * N1W * C::ZS + pb_k2;
      float2 u[N1W];
      sfor<0, N1W>([&](auto D) { u[D] = col[(N1W - 1 - D) * C::ZS]; });
      row_levels<N1W>(u, tw.w1);
      if (g.scale != 1.0f) {
        sfor<0, N1W>([&](auto K) { u[K] = make_float2(u[K].x * g.scale, u[K].y * g.scale); });
      }
      sfor<0, N1W>([&](auto K) { col[K * C::ZS] = u[K]; });
    });
  };

  // Rotated loop as in the 2D kernel: the loads of chunk c+1 are issued
  // before the column phase of chunk c.
  load_chunk(row0);
  plane_phase();
  __syncthreads();
  const float2* zcol = zl + (cp_c * N1W + cp_k1) * C::ZS + cp_k2;
  for (int c = 0; c < nchunks; ++c) {
    const int64_t crow = row0 + (int64_t)c * C::CR;
    if (c + 1 < nchunks) load_chunk(crow + C::CR);
    __builtin_amdgcn_sched_barrier(0);

    // step st writes window row q0 = crow + st - (n0 - 1) if it lies in the slab
    const tree::StepSpan sp = tree::step_span(crow, row0, q0_end, N0W - 1, C::CR);
    uint64_t row_addr = tree::uniform_u64((uint64_t)(uintptr_t)ystrip +
                                          (uint64_t)(crow - (N0W - 1)) * row_bytes);
    // In the slab's first chunk step st is the slab's row st: its priming
    // steps (st < n0 - 1) compute only the axis-0 levels the slab's windows
    // use (column_levels, as in the 2D kernel).
    auto run_steps = [&](auto FIRST) __attribute__((always_inline)) {
      sfor<0, C::CR>([&](auto STc) {
        constexpr int st = STc;
        const float2 z = zcol[st * C::ZROW];
        const auto out = tree::step_rsrc(row_addr, st, sp, strip_bytes);
        row_addr += row_bytes;
        column_levels<N0W, 1, st % C::RING, (FIRST ? st : -1)>(
            z, ring, lanefac, lw, tw.w0, [&](auto J, float2 v) {
              store_buf<C::NT_STORES>(out, lane_off + J * C::NK * (int)sizeof(float2), v);
            });
      });
    };
    if (c == 0) {
      run_steps(std::true_type{});
    } else {
      run_steps(std::false_type{});
    }
    __syncthreads();
    if (c + 1 < nchunks) {
      plane_phase();
      __syncthreads();
    }
  }
}

template <int N0W, int N1W, int N2W, bool REAL>
__global__ __launch_bounds__(64) void tree3_fwd_kernel(const void* __restrict__ xv,
                                                       float2* __restrict__ y, Tree3Geom g,
                                                       Twiddles3F32 tw) {
  using C = Tree3Cfg<N0W, N1W, N2W, REAL>;
  __shared__ float2 zl[C::LDS_FLOAT2];
  int id = g.order ? (int)blockIdx.x : tree::xcd_tile(blockIdx.x, gridDim.x);
  const int strip = id % g.nstrips;
  id /= g.nstrips;
  const int q1 = (int)(id % g.P1);
  id /= (int)g.P1;
  const int slab = id % g.nslabs;
  const int b = id / g.nslabs;
  tree3_fwd_tile<N0W, N1W, N2W, REAL>(xv, y, g, tw, strip, q1, slab, b, zl);
}

template <int N0W, int N1W, int N2W, bool REAL>
hipError_t launch3_one(const void* x, float2* y, const Tree3Geom& g, const Twiddles3F32& tw,
                       hipStream_t stream) {
  using C = Tree3Cfg<N0W, N1W, N2W, REAL>;
  const int64_t nb = (int64_t)g.batch * g.nslabs * g.P1 * g.nstrips;
  const unsigned pad =
      tree::occupancy_lds(g.wpc, g.lds_cu, C::LDS_FLOAT2 * (unsigned)sizeof(float2));
  hipLaunchKernelGGL((tree3_fwd_kernel<N0W, N1W, N2W, REAL>), dim3((unsigned)nb), dim3(64), pad,
                     stream, x, y, g, tw);
  return hipGetLastError();
}

// One translation unit per (n0, input type) instantiates every (n1, n2).
template <int N0W, bool REAL>
hipError_t launch3_n0(int n1, int n2, const void* x, float2* y, const Tree3Geom& g,
                      const Twiddles3F32& tw, hipStream_t s) {
  switch (n1 * 16 + n2) {
    case 2 * 16 + 2: return launch3_one<N0W, 2, 2, REAL>(x, y, g, tw, s);
    case 2 * 16 + 4: return launch3_one<N0W, 2, 4, REAL>(x, y, g, tw, s);
    case 2 * 16 + 8: return launch3_one<N0W, 2, 8, REAL>(x, y, g, tw, s);
    case 4 * 16 + 2: return launch3_one<N0W, 4, 2, REAL>(x, y, g, tw, s);
    case 4 * 16 + 4: return launch3_one<N0W, 4, 4, REAL>(x, y, g, tw, s);
    case 4 * 16 + 8: return launch3_one<N0W, 4, 8, REAL>(x, y, g, tw, s);
    case 8 * 16 + 2: return launch3_one<N0W, 8, 2, REAL>(x, y, g, tw, s);
    case 8 * 16 + 4: return launch3_one<N0W, 8, 4, REAL>(x, y, g, tw, s);
    case 8 * 16 + 8: return launch3_one<N0W, 8, 8, REAL>(x, y, g, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tree3

#define SWDFT_FWD3_DECL(N0W, TAG)                                                             \
  hipError_t launch_tree3_fwd_n0_##N0W##_##TAG(int, int, const void*, float2*, const Tree3Geom&, \
                                               const Twiddles3F32&, hipStream_t);
SWDFT_FWD3_DECL(2, r)
SWDFT_FWD3_DECL(2, c)
SWDFT_FWD3_DECL(4, r)
SWDFT_FWD3_DECL(4, c)
SWDFT_FWD3_DECL(8, r)
SWDFT_FWD3_DECL(8, c)
SWDFT_FWD3_DECL(16, r)
SWDFT_FWD3_DECL(16, c)
#undef SWDFT_FWD3_DECL

}  // namespace swdft
