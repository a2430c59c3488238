// Streaming 2D Tree SWDFT for gfx950: the order of Sec. 4.3 in which the
// loops over trees are innermost and rows arrive one after another. The
// column levels (Eq. (6)) of a stream only need level u-1 of the last
// s_u = n0/2^u trees; that state (the 2^(u-1) nodes of each of those trees,
// m0 n0 / 2 complex values per (q1, k1) stream) stays resident in device
// memory between calls, so each new input row
// costs the 2(n0-1) node operations per stream of Eq. (8) and completes one
// row of P1 windows as soon as it arrives.
//
// One wave owns QW = 64/(n1 KG) window columns (streams split over KG = 2
// lanes from n0 = 4 on) and processes the R
// rows of one call: the row levels (Eq. (5)) per position into LDS (inputs
// loaded a chunk ahead), then the column levels with the rings loaded from,
// and at the end saved to, the resident state. The state is kept in absolute
// row order: the nodes of tree p at level u-1 sit in tree slot (p mod s_u).
// The unrolled column phase uses static ring slots (relative step mod s_u),
// so the load and the save rotate by (first row mod s_u) through computed
// memory addresses. Steps past the call's last row are skipped (a
// wave-uniform branch), so calls may carry any number of rows.
#pragma once

#include "tree_fwd_kernel.h"

namespace swdft {
namespace tree {

// Lanes per column stream: two from n0 = 4 on (the split of the single-image
// kernel), which doubles the strips of a call and halves each lane's column
// work per row; calls are short, so their time is set by how long one wave
// takes for its rows.
constexpr int stream_kg(int n0) { return n0 >= 4 ? 2 : 1; }

template <int N0W, int N1W, bool REAL>
__global__ __launch_bounds__(64) void tree_stream_kernel(const void* __restrict__ xv,
                                                         float2* __restrict__ y,
                                                         float2* __restrict__ state, StreamGeom g,
                                                         TwiddlesF32 tw) {
  constexpr int KG = stream_kg(N0W);
  using C = TreeCfg<N0W, N1W, REAL, KG>;
  using CC = ColCfg<N0W, KG>;
  __shared__ float2 zl[C::LDS_FLOAT2];
  const int lane = threadIdx.x;
  const int strip = blockIdx.x;
  const StreamGeom sg = uniform_copy(g);
  const float2* w0 = tw.w0;
  const float2* w1 = tw.w1;

  const int64_t q1_0 = (int64_t)strip * C::QW;
  const int64_t p_start = sg.rows_before;  // absolute index of the call's first row
  const int64_t R = sg.rows;
  const int nchunks = (int)((R + C::CR - 1) / C::CR);
  // first window row this call completes (windows end at row q0 + n0 - 1)
  const int64_t q0_first = max((int64_t)0, p_start - (N0W - 1));

  using XT = std::conditional_t<REAL, float, float2>;
  const XT* x = reinterpret_cast<const XT*>(xv);  // the call's first row

  // row-phase roles: lane (r, c)
  const int rp_r = lane / C::QW;
  const int rp_c = lane % C::QW;
  const int64_t rp_q1 = q1_0 + rp_c;
  // column-phase roles: lane (c, residue, k1)
  const int cp_c = lane / (N1W * KG);
  const int cp_res = (lane / N1W) % KG;
  const int cp_k1 = lane % N1W;
  float2* ystrip = y + q1_0 * (N0W * N1W);
  const uint64_t row_bytes = (uint64_t)sg.P1 * (N0W * N1W * sizeof(float2));
  const uint32_t strip_bytes = uniform_u32(
      (uint32_t)(min((int64_t)C::QW, sg.P1 - q1_0) * (N0W * N1W * (int)sizeof(float2))));
  const uint32_t lane_off =
      (uint32_t)((cp_c * (N0W * N1W) + cp_res * N1W + cp_k1) * (int)sizeof(float2));

  // resident state: slot k of this lane at state[k * state_stride + strip * 64 + lane]
  float2* st_lane = state + (int64_t)strip * 64 + lane;
  const int64_t state_stride = (int64_t)sg.nstrips * 64;

  // per-lane twiddle factors of a split stream (as in the single-image kernel)
  float2 lanefac[CC::M0 + 1];
  float2 lw[CC::M0 + 1][CC::LW];
  lanefac[0] = make_float2(1.f, 0.f);
  sfor<1, CC::M0 + 1>([&](auto U) {
    constexpr int u = U;
    if constexpr (KG > 1) {
      lanefac[u] = w0[(cp_res & ((1 << u) - 1)) * (N0W >> u)];
    } else {
      lanefac[u] = make_float2(1.f, 0.f);
    }
  });
  sfor<1, CC::M0 + 1>([&](auto U) {
    constexpr int u = U;
    sfor<0, CC::LW>([&](auto J) {
      constexpr int j = J;
      if constexpr (CC::folded(u, j)) lw[u][j] = cmul(lanefac[u], uload(w0 + CC::tw_index(u, j)));
    });
  });

  // ring of level u-1: s_u tree slots of held(u-1) nodes each; static tree
  // slot t holds the tree whose absolute row index is congruent to
  // p_start + t modulo s_u
  float2 ring[CC::RING_TOTAL];
  auto state_index = [&](int u, int s, int hp, int t, int j) {
    return (int64_t)(CC::ring_off(u) + (int)((p_start + t) % s) * hp + j) * state_stride;
  };
  sfor<1, CC::M0 + 1>([&](auto U) {
    constexpr int u = U;
    constexpr int s = N0W >> u;
    constexpr int hp = CC::held(u - 1);
    sfor<0, s>([&](auto T) {
      sfor<0, hp>([&](auto J) {
        ring[CC::ring_off(u) + T * hp + J] = st_lane[state_index(u, s, hp, T, J)];
      });
    });
  });

  // Inputs of one chunk (rows rel_c + ps * R + r of the call) through a buffer
  // resource over the call's rows: rows past the call and columns past the
  // image edge read zero (Sec. 4.7). Loaded a chunk ahead, so that their
  // latency hides behind the previous chunk's column phase.
  constexpr int EB = (int)sizeof(XT);
  uint32_t x_off[N1W];
  sfor<0, N1W>([&](auto D) {
    constexpr int d = D;
    const int64_t col = rp_q1 + (N1W - 1 - d);
    x_off[d] = col < sg.N1 ? (uint32_t)(((int64_t)rp_r * sg.N1 + col) * EB) : kOutOfRange;
  });
  constexpr int PASSES = C::CR / C::R;
  XT xin[PASSES][N1W];
  auto load_chunk = [&](int64_t rel_c) __attribute__((always_inline)) {
    const int64_t rows = min((int64_t)C::CR, R - rel_c);
    const auto rs = buf_rsrc(x + (rows > 0 ? rel_c : 0) * sg.N1,
                             rows > 0 ? (uint32_t)(rows * sg.N1 * EB) : 0u);
    sfor<0, PASSES>([&](auto PS) {
      constexpr int ps = PS;
      sfor<0, N1W>([&](auto D) {
        constexpr int d = D;
        xin[ps][d] = load_buf<REAL>(rs, x_off[d] + (uint32_t)(ps * C::R * sg.N1 * EB));
      });
    });
  };
  // ---- row phase: CR rows x QW window columns of Z into LDS
  auto row_phase = [&]() __attribute__((always_inline)) {
    sfor<0, PASSES>([&](auto PS) {
      constexpr int ps = PS;
      float2 v[N1W];
      sfor<0, N1W>([&](auto D) {
        if constexpr (REAL) {
          v[D] = make_float2(xin[ps][D], 0.f);
        } else {
          v[D] = xin[ps][D];
        }
      });
      row_levels<N1W>(v, w1);
      if (sg.scale != 1.0f) {
        sfor<0, N1W>([&](auto K) { v[K] = make_float2(v[K].x * sg.scale, v[K].y * sg.scale); });
      }
      float2* zrow = zl + (ps * C::R + rp_r) * C::ZROW + rp_c * C::ZS;
      sfor<0, N1W>([&](auto K) { zrow[K] = v[K]; });
    });
  };

  load_chunk(0);
  row_phase();
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int64_t rel0 = (int64_t)c * C::CR;  // relative index of the chunk's first row
    load_chunk(rel0 + C::CR);  // past the call's rows: zeros, no memory touched
    __builtin_amdgcn_sched_barrier(0);

    // ---- column phase: the chunk's rows that this call carries. Step st
    // completes window row q0 = p_start + rel0 + st - (n0 - 1) when q0 >= 0;
    // row_addr is the address of that row of step 0 (an integer: it may lie
    // before y).
    const int64_t crow = p_start + rel0;
    const StepSpan sp = step_span(crow, 0, crow + C::CR, N0W - 1, C::CR);
    uint64_t row_addr = uniform_u64((uint64_t)(uintptr_t)ystrip +
                                    (uint64_t)(crow - (N0W - 1) - q0_first) * row_bytes);
    sfor<0, C::CR>([&](auto STc) {
      constexpr int st = STc;
      const auto out = step_rsrc(row_addr, st, sp, strip_bytes);
      row_addr += row_bytes;
      if (rel0 + st < R) {
        const float2 z = zl[st * C::ZROW + cp_c * C::ZS + cp_k1];
        // Non-temporal stores for every n1. Plain stores for the narrow rows
        // of n1 < 16, which help the long single-plan launches, measured
        // slower for these short calls (1024-wide rows in 64-row pushes,
        // 8 x 8: 295 -> 330 us per pass; 16 x 8: 469 -> 499 us).
        if constexpr (N0W == 1) {
          store_buf_nt(out, lane_off, z);
        } else {
          column_levels<N0W, KG, st % C::RING>(z, ring, lanefac, lw, w0, [&](auto J, float2 v) {
            store_buf_nt(out, lane_off + (KG * J) * N1W * (int)sizeof(float2), v);
          });
        }
      }
    });
    __syncthreads();
    if (c + 1 < nchunks) {
      row_phase();
      __syncthreads();
    }
  }

  // save the rings in absolute order (the same rotation as the load)
  sfor<1, CC::M0 + 1>([&](auto U) {
    constexpr int u = U;
    constexpr int s = N0W >> u;
    constexpr int hp = CC::held(u - 1);
    sfor<0, s>([&](auto T) {
      sfor<0, hp>([&](auto J) {
        st_lane[state_index(u, s, hp, T, J)] = ring[CC::ring_off(u) + T * hp + J];
      });
    });
  });
}

template <int N0W, int N1W, bool REAL>
hipError_t launch_stream_one(const void* x, float2* y, float2* state, const StreamGeom& g,
                             const TwiddlesF32& tw, hipStream_t stream) {
  static_assert(64 % (N1W * stream_kg(N0W)) == 0, "a wave holds whole split streams");
  hipLaunchKernelGGL((tree_stream_kernel<N0W, N1W, REAL>), dim3((unsigned)g.nstrips), dim3(64), 0,
                     stream, x, y, state, g, tw);
  return hipGetLastError();
}

template <int N0W, bool REAL>
hipError_t launch_stream_n0(int n1, const void* x, float2* y, float2* state, const StreamGeom& g,
                            const TwiddlesF32& tw, hipStream_t s) {
  switch (n1) {
    case 1: return launch_stream_one<N0W, 1, REAL>(x, y, state, g, tw, s);
    case 2: return launch_stream_one<N0W, 2, REAL>(x, y, state, g, tw, s);
    case 4: return launch_stream_one<N0W, 4, REAL>(x, y, state, g, tw, s);
    case 8: return launch_stream_one<N0W, 8, REAL>(x, y, state, g, tw, s);
    case 16: return launch_stream_one<N0W, 16, REAL>(x, y, state, g, tw, s);
    case 32: return launch_stream_one<N0W, 32, REAL>(x, y, state, g, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tree

#define SWDFT_STREAM_DECL(N0W, TAG)                                                            \
  hipError_t launch_tree_stream_n0_##N0W##_##TAG(int, const void*, float2*, float2*,            \
                                                 const StreamGeom&, const TwiddlesF32&, hipStream_t);
SWDFT_STREAM_DECL(1, r)
SWDFT_STREAM_DECL(1, c)
SWDFT_STREAM_DECL(2, r)
SWDFT_STREAM_DECL(2, c)
SWDFT_STREAM_DECL(4, r)
SWDFT_STREAM_DECL(4, c)
SWDFT_STREAM_DECL(8, r)
SWDFT_STREAM_DECL(8, c)
SWDFT_STREAM_DECL(16, r)
SWDFT_STREAM_DECL(16, c)
SWDFT_STREAM_DECL(32, r)
SWDFT_STREAM_DECL(32, c)
#undef SWDFT_STREAM_DECL

}  // namespace swdft
