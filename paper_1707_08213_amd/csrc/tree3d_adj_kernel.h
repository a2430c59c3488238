// Adjoint of the 3D Tree SWDFT for gfx950 (the k-dimensional extension of
// Sec. 4.4, k = 3): dx = M^H dy, M the linear map x -> y of the 3D forward
// transform (three level equations instantiating Eq. (7)).
//
// M is a product of level maps; its adjoint runs the transposed levels in
// reverse order, as the 2D adjoint does (tree_adj_kernel.h):
//  * axis 0, streamed UP a slab of window rows: the transposed column levels
//    of the 2D adjoint with the node index running over (k1, k2) pairs (lane
//    (c, k1, k2) reads dy[q0][q1][q2_0 + c][k0][k1][k2] for every k0), which
//    leave dZ[p0][c][k1][k2], the cotangent of the (n1 x n2) DFTs of the plane
//    patches, in LDS;
//  * the plane phase transposed, per chunk of planes: pass B^T runs the
//    transposed axis-1 levels on the n1 bins of each (c, k2) column, pass A^T
//    the transposed axis-2 levels on the n2 bins of each (c, j1) line; the
//    result is the contribution of window (q1, q2_0 + c) to x[p0][q1 + j1]
//    [q2_0 + c + j2], j1 < n1, j2 < n2;
//  * overlap-add of the strip's QW windows along axis 2 (QW + n2 - 1 x columns
//    per axis-1 line), written to a workspace per tile (window row q1, strip);
//    a second kernel adds, per dx element, the partials of the n1 window rows
//    q1 and the strips that cover it, in a fixed order (deterministic, no
//    atomics).
// Window rows that do not exist (q0 outside [0, P0), the incomplete trees of
// Sec. 4.7) contribute nothing: their dy rows read zero.
#pragma once

#include "tree3d_fwd_kernel.h"
#include "tree_adj_kernel.h"

namespace swdft {
namespace tree3 {

using tree::cadd;
using tree::load_buf_nt;
using tree::row_levels_adj;
using tree::StepSpan;
using tree::step_rsrc;
using tree::uniform_u32;
using tree::uniform_u64;

template <int N0W, int N1W, int N2W>
struct Adj3Cfg {
  static constexpr int NK = N1W * N2W;
  static constexpr int QW = 64 / NK;                       // windows per strip (axis 2)
  static constexpr int RING = N0W > 1 ? N0W / 2 : 1;
  static constexpr int PF = N0W <= 8 ? 4 : 2;             // dy rows in flight
  static constexpr int RA = N2W;                           // plane rows per pass A^T
  static constexpr int RB = N1W;                           // plane rows per pass B^T
  static constexpr int CR0 = RA > RB ? RA : RB;
  static constexpr int CR1 = CR0 > RING ? CR0 : RING;
  static constexpr int CR = CR1 > PF ? CR1 : PF;          // plane rows per chunk
  static constexpr int PA = CR / RA;
  static constexpr int PB = CR / RB;
  static constexpr int ZS = N2W + 1;                       // padded (c, j1) line in LDS
  static constexpr int ZROW = QW * N1W * ZS;               // float2 per plane row
  static constexpr int WCOLS = QW + N2W - 1;               // x columns (axis 2) of a strip
  static constexpr int WROW = N1W * WCOLS;                 // workspace values per plane
  static_assert(NK <= 64 && 64 % NK == 0, "one wave holds the (k1, k2) plane of a window");
  static_assert(CR % RING == 0 && CR % PF == 0 && CR % RA == 0 && CR % RB == 0,
                "chunks start on ring periods and prefetch slots");
};

template <int N0W, int N1W, int N2W, bool REAL>
__global__ __launch_bounds__(64) void tree3_adj_kernel(const float2* __restrict__ dy,
                                                       void* __restrict__ wsv, Adj3Geom g,
                                                       Twiddles3F32 tw) {
  using C = Adj3Cfg<N0W, N1W, N2W>;
  using CC = tree::ColCfg<N0W, 1>;
  __shared__ float2 zl[C::CR * C::ZROW];

  const int lane = threadIdx.x;
  int id = tree::xcd_tile(blockIdx.x, gridDim.x);
  const int strip = id % g.nstrips;
  id /= g.nstrips;
  const int q1 = (int)(id % g.P1);
  id /= (int)g.P1;
  const int slab = id % g.nslabs;
  const int b = id / g.nslabs;

  const int64_t q2_0 = (int64_t)strip * C::QW;
  const int64_t r0 = (int64_t)slab * g.S;            // first dx plane of the slab
  const int64_t r1 = min(r0 + (int64_t)g.S, g.N0);   // one past the last
  // positions run from p_top down to r0; p_top + 1 is a multiple of CR, so
  // the ring slots of every step are known at compile time
  const int64_t p_hi = r1 + N0W - 2;
  const int nchunks = (int)((p_hi - r0 + 1 + C::CR - 1) / C::CR);
  const int64_t p_top = r0 + (int64_t)nchunks * C::CR - 1;
  const int64_t q0_last = min(r1 - 1, g.P0 - 1);     // last window row read by this slab

  // column-phase roles: lane (c, k1, k2)
  const int cp_c = lane / C::NK;
  const int cp_k = lane % C::NK;
  const int cp_k1 = cp_k / N2W;
  const int cp_k2 = cp_k % N2W;
  const float2* dystrip =
      dy + b * g.y_image_stride + ((int64_t)q1 * g.P2 + q2_0) * (N0W * C::NK);
  const uint64_t row_bytes = (uint64_t)g.P1 * g.P2 * (N0W * C::NK * sizeof(float2));
  const uint32_t strip_bytes = uniform_u32(
      (uint32_t)(min((int64_t)C::QW, g.P2 - q2_0) * (N0W * C::NK * (int)sizeof(float2))));
  const uint32_t lane_off = (uint32_t)((cp_c * (N0W * C::NK) + cp_k) * (int)sizeof(float2));
  // pass roles
  const int pa_j1 = lane % N1W;
  const int pa_c = (lane / N1W) % C::QW;
  const int pa_r = lane / (N1W * C::QW);
  const int pb_k2 = lane % N2W;
  const int pb_c = (lane / N2W) % C::QW;
  const int pb_r = lane / (N2W * C::QW);

  float2 lanefac[CC::M0 + 1];
  float2 lwc[CC::M0 + 1][CC::LW];
  sfor<0, CC::M0 + 1>([&](auto U) { lanefac[U] = make_float2(1.f, 0.f); });
  auto no_partner = [](float2 v) { return v; };  // streams are not split across lanes

  float2 ring[CC::RING_TOTAL];
  sfor<0, CC::RING_TOTAL>([&](auto K) { ring[K] = make_float2(0.f, 0.f); });

  // dy rows in step order gstep = 0, 1, ...: position p = p_top - gstep,
  // window row q0 = p - (n0 - 1); rows outside [0, q0_last] (or p < r0) read
  // zeros through an empty resource. The row address is a running scalar.
  const int64_t g_first = p_top - (N0W - 1) - q0_last;
  const int64_t g_last = min(p_top - (N0W - 1), p_top - r0);
  const int64_t g_lo = g_first > 0 ? g_first : 0;
  const StepSpan lsp{(int)uniform_u32((uint32_t)g_lo),
                     uniform_u32((uint32_t)(g_last >= g_lo ? g_last - g_lo + 1 : 0))};
  uint64_t dy_addr = uniform_u64((uint64_t)(uintptr_t)dystrip +
                                 (uint64_t)(p_top - (N0W - 1)) * row_bytes);
  int gstep = 0;
  auto load_step = [&](float2 (&dst)[N0W]) {
    const auto rs = step_rsrc(dy_addr, gstep, lsp, strip_bytes);
    sfor<0, N0W>([&](auto K) { dst[K] = load_buf_nt(rs, lane_off + K * C::NK * (int)sizeof(float2)); });
    dy_addr -= row_bytes;
    ++gstep;
  };
  float2 pf[C::PF][N0W];
  sfor<0, C::PF>([&](auto S) { load_step(pf[S]); });

  float* wsr = reinterpret_cast<float*>(wsv);
  float2* wsc = reinterpret_cast<float2*>(wsv);
  // workspace rows of this tile: [b][q1][strip][plane][j1][col]
  const int64_t ws_tile = (((int64_t)b * g.P1 + q1) * g.nstrips + strip) * g.N0;

  for (int c = 0; c < nchunks; ++c) {
    const int64_t cbase = (int64_t)c * C::CR;
    // chunk planes p = p_top - cbase - st; LDS row st holds dZ[p]
    sfor<0, C::CR>([&](auto STc) {
      constexpr int st = STc;
      constexpr int slot = st % C::PF;
      constexpr int pm = (C::RING - 1 - (st % C::RING));
      float2 gcur[N0W];
      sfor<0, N0W>([&](auto K) { gcur[K] = pf[slot][K]; });
      load_step(pf[slot]);
      float2 dz;
      if constexpr (N0W == 1) {
        dz = gcur[0];
      } else {
        dz = tree::column_levels_adj<N0W, 1, pm>(gcur, ring, lanefac, lwc, tw.w0, false,
                                                 no_partner);
      }
      zl[st * C::ZROW + (cp_c * N1W + cp_k1) * C::ZS + cp_k2] = dz;
    });
    __syncthreads();
    // pass B^T: transposed axis-1 levels per (plane row, window, k2) column;
    // the forward read the line of j1 = n1 - 1 - d into position d
    sfor<0, C::PB>([&](auto P) {
      constexpr int pb = P;
      float2* col = zl + (pb * C::RB + pb_r) * C::ZROW + pb_c * N1W * C::ZS + pb_k2;
      float2 u[N1W];
      sfor<0, N1W>([&](auto K) { u[K] = col[K * C::ZS]; });
      row_levels_adj<N1W>(u, tw.w1);
      sfor<0, N1W>([&](auto D) { col[(N1W - 1 - D) * C::ZS] = u[D]; });
    });
    __syncthreads();
    // pass A^T: transposed axis-2 levels per (plane row, window, j1) line;
    // v[d] is the cotangent of x at column c + n2 - 1 - d of the strip,
    // stored in place at column offset n2 - 1 - d
    sfor<0, C::PA>([&](auto P) {
      constexpr int pa = P;
      float2* line = zl + (pa * C::RA + pa_r) * C::ZROW + (pa_c * N1W + pa_j1) * C::ZS;
      float2 v[N2W];
      sfor<0, N2W>([&](auto K) { v[K] = line[K]; });
      row_levels_adj<N2W>(v, tw.w2);
      // (windows past the strip's edge read dy = 0 and contribute 0)
      sfor<0, N2W>([&](auto K) { line[K] = v[N2W - 1 - K]; });
    });
    __syncthreads();
    // overlap-add the strip's windows along axis 2 for each (plane, j1) line
    for (int o = lane; o < C::CR * C::WROW; o += 64) {
      const int srow = o / C::WROW;
      const int j1 = (o / C::WCOLS) % N1W;
      const int col = o % C::WCOLS;
      const int64_t prow = p_top - cbase - srow;
      float2 acc = make_float2(0.f, 0.f);
      const int c_lo = col - (N2W - 1) > 0 ? col - (N2W - 1) : 0;
      const int c_hi = col < C::QW - 1 ? col : C::QW - 1;
      for (int cc = c_lo; cc <= c_hi; ++cc)
        acc = cadd(acc, zl[srow * C::ZROW + (cc * N1W + j1) * C::ZS + (col - cc)]);
      if (prow >= r0 && prow < r1) {
        const int64_t idx = (ws_tile + prow) * C::WROW + j1 * C::WCOLS + col;
        if constexpr (REAL) {
          wsr[idx] = acc.x * g.scale;
        } else {
          wsc[idx] = make_float2(acc.x * g.scale, acc.y * g.scale);
        }
      }
    }
    __syncthreads();
  }
}

// dx[b][v0][v1][v2] = sum over window rows a in [v1 - n1 + 1, v1] of axis 1
// and strips s whose x columns [s*QW, s*QW + QW + n2 - 1) contain v2 of
// ws[b][a][s][v0][v1 - a][v2 - s*QW], in ascending (a, s). One workgroup per
// (volume line (b, v0, v1), block of columns v2).
template <int N1W, int N2W, bool REAL>
__global__ __launch_bounds__(tree::kAdjReduceThreads) void tree3_adj_reduce_kernel(
    const void* __restrict__ wsv, void* __restrict__ dxv, Adj3Geom g, int cblocks) {
  constexpr int QW = 64 / (N1W * N2W);
  constexpr int WCOLS = QW + N2W - 1;
  constexpr int WROW = N1W * WCOLS;
  const int64_t line = (int64_t)blockIdx.x / cblocks;  // (b * N0 + v0) * N1 + v1
  const int cb = (int)(blockIdx.x - line * cblocks);
  const int64_t v2 = (int64_t)cb * tree::kAdjReduceThreads + threadIdx.x;
  if (v2 >= g.N2) return;
  const int64_t v1 = line % g.N1;
  const int64_t bv0 = line / g.N1;
  const int64_t v0 = bv0 % g.N0;
  const int64_t b = bv0 / g.N0;
  int64_t a_lo = v1 - (N1W - 1);
  a_lo = a_lo > 0 ? a_lo : 0;
  const int64_t a_hi = v1 < g.P1 - 1 ? v1 : g.P1 - 1;
  int64_t s_lo = v2 - (WCOLS - 1);
  s_lo = s_lo > 0 ? (s_lo + QW - 1) / QW : 0;
  int64_t s_hi = v2 / QW;
  if (s_hi > g.nstrips - 1) s_hi = g.nstrips - 1;
  float2 acc = make_float2(0.f, 0.f);
  for (int64_t a = a_lo; a <= a_hi; ++a) {
    for (int64_t s = s_lo; s <= s_hi; ++s) {
      const int64_t idx = ((((b * g.P1 + a) * g.nstrips + s) * g.N0 + v0) * WROW) +
                          (v1 - a) * WCOLS + (v2 - s * QW);
      if constexpr (REAL) {
        acc.x += reinterpret_cast<const float*>(wsv)[idx];
      } else {
        acc = cadd(acc, reinterpret_cast<const float2*>(wsv)[idx]);
      }
    }
  }
  const int64_t out = line * g.N2 + v2;
  if constexpr (REAL) {
    reinterpret_cast<float*>(dxv)[out] = acc.x;
  } else {
    reinterpret_cast<float2*>(dxv)[out] = acc;
  }
}

template <int N0W, int N1W, int N2W, bool REAL>
hipError_t launch3_adj_one(const float2* dy, void* ws, void* dx, const Adj3Geom& g,
                           const Twiddles3F32& tw, hipStream_t stream) {
  using C = Adj3Cfg<N0W, N1W, N2W>;
  const int64_t nb = (int64_t)g.batch * g.nslabs * g.P1 * g.nstrips;
  const unsigned pad =
      tree::occupancy_lds(g.wpc, g.lds_cu, C::CR * C::ZROW * (unsigned)sizeof(float2));
  hipLaunchKernelGGL((tree3_adj_kernel<N0W, N1W, N2W, REAL>), dim3((unsigned)nb), dim3(64), pad,
                     stream, dy, ws, g, tw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int cblocks = (int)((g.N2 + tree::kAdjReduceThreads - 1) / tree::kAdjReduceThreads);
  hipLaunchKernelGGL((tree3_adj_reduce_kernel<N1W, N2W, REAL>),
                     dim3((unsigned)((int64_t)g.batch * g.N0 * g.N1 * cblocks)),
                     dim3(tree::kAdjReduceThreads), 0, stream, ws, dx, g, cblocks);
  return hipGetLastError();
}

// One translation unit per (n0, input type) instantiates every (n1, n2).
template <int N0W, bool REAL>
hipError_t launch3_adj_n0(int n1, int n2, const float2* dy, void* ws, void* dx,
                          const Adj3Geom& g, const Twiddles3F32& tw, hipStream_t s) {
  switch (n1 * 16 + n2) {
    case 2 * 16 + 2: return launch3_adj_one<N0W, 2, 2, REAL>(dy, ws, dx, g, tw, s);
    case 2 * 16 + 4: return launch3_adj_one<N0W, 2, 4, REAL>(dy, ws, dx, g, tw, s);
    case 2 * 16 + 8: return launch3_adj_one<N0W, 2, 8, REAL>(dy, ws, dx, g, tw, s);
    case 4 * 16 + 2: return launch3_adj_one<N0W, 4, 2, REAL>(dy, ws, dx, g, tw, s);
    case 4 * 16 + 4: return launch3_adj_one<N0W, 4, 4, REAL>(dy, ws, dx, g, tw, s);
    case 4 * 16 + 8: return launch3_adj_one<N0W, 4, 8, REAL>(dy, ws, dx, g, tw, s);
    case 8 * 16 + 2: return launch3_adj_one<N0W, 8, 2, REAL>(dy, ws, dx, g, tw, s);
    case 8 * 16 + 4: return launch3_adj_one<N0W, 8, 4, REAL>(dy, ws, dx, g, tw, s);
    case 8 * 16 + 8: return launch3_adj_one<N0W, 8, 8, REAL>(dy, ws, dx, g, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tree3

#define SWDFT_ADJ3_DECL(N0W, TAG)                                                             \
  hipError_t launch_tree3_adj_n0_##N0W##_##TAG(int, int, const float2*, void*, void*,          \
                                               const Adj3Geom&, const Twiddles3F32&, hipStream_t);
SWDFT_ADJ3_DECL(2, r)
SWDFT_ADJ3_DECL(2, c)
SWDFT_ADJ3_DECL(4, r)
SWDFT_ADJ3_DECL(4, c)
SWDFT_ADJ3_DECL(8, r)
SWDFT_ADJ3_DECL(8, c)
SWDFT_ADJ3_DECL(16, r)
SWDFT_ADJ3_DECL(16, c)
#undef SWDFT_ADJ3_DECL

}  // namespace swdft
