// Adjoint of the 2D Tree SWDFT for gfx950: dx = M^H dy, where M is the
// linear map x -> y of the forward transform (Eq. (2), computed by the
// levels of Eq. (5)-(6)).
//
// The forward map is a product of level maps; its adjoint is the product of
// the transposed level maps in reverse order. For a column level u (shift
// s = n0/2^u, h = 2^{u-1}, w_i = Omega0[i s]) the forward node pair
//   T_u[p][i] = T_{u-1}[p-s][i] + w_i T_{u-1}[p][i],  T_u[p][i+h] = T_{u-1}[p-s][i] - w_i T_{u-1}[p][i]
// transposes to
//   G_{u-1}[p][i] = (G_u[p+s][i] + G_u[p+s][i+h]) + conj(w_i) (G_u[p][i] - G_u[p][i+h]),
// so the column adjoint streams UP the image (descending p) and keeps, per
// level, the pair sums S_u[p][i] = G_u[p][i] + G_u[p][i+h] of the last s
// positions in a register ring: the same n0/2 values per level as the
// forward ring. G_{m0}[p] is dy of the window whose last row is p (zero where
// that window does not exist, which also gives the incomplete trees of
// Sec. 4.7 zero gradient), and G_0[p] = dZ[p], the cotangent of the row DFTs.
//
// The row adjoint transposes the per-position row levels: from dZ[q1][k1] it
// forms the contribution of window column q1 to x[p0][q1 .. q1+n1-1] (an
// unnormalised inverse DFT computed by the transposed levels), and adds the
// contributions of the window columns of the wave's strip (overlap-add).
//
// Mapping: like the forward kernel, one wave owns QW = 64/n1 window columns
// and a slab of output rows of dx. Lane (c, k1) reads dy[q0][q1][k0][k1] for
// all k0 (each load instruction covers whole 128-byte lines), PF steps ahead
// of use (register prefetch) so a wave keeps PF rows of loads in flight.
// The slab is primed by the n0-1 window rows below it. A strip's row adjoint
// covers x columns [q1_0, q1_0 + QW + n1 - 1); columns near strip edges get
// parts from neighbouring strips, so each wave writes its partial sums for
// its QW + n1 - 1 columns to a workspace and a second small kernel adds the
// at most ceil((QW+n1-1)/QW) partials of each dx element in a fixed order
// (deterministic, no atomics). dy is read once per slab (plus the priming
// rows); everything else stays on chip.
#pragma once
#include <type_traits>

#include "tree_fwd_kernel.h"

namespace swdft {
namespace tree {

// conj(Omega[IDX]) * d for IDX < N/2 known at compile time.
template <int IDX, int N>
__device__ __forceinline__ float2 twmul_conj(float2 d, const float2* w) {
  if constexpr (IDX == 0) {
    return d;
  } else if constexpr (4 * IDX == N) {
    return make_float2(-d.y, d.x);  // conj(-i) = i
  } else {
    const float2 t = uload(w + IDX);
    return make_float2(t.x * d.x + t.y * d.y, t.x * d.y - t.y * d.x);
  }
}

// Transposed row levels t = m1..1 for one tree position p. On entry
// v[k1] = dZ[k1]; on exit v[d] is the cotangent of x[p - d], d < n1.
template <int N1W>
__device__ __forceinline__ void row_levels_adj(float2 (&v)[N1W], const float2* w1) {
  constexpr int M1 = ilog2(N1W);
  sfor<0, M1>([&](auto V) {
    constexpr int t = M1 - V;  // M1 .. 1
    constexpr int s = N1W >> t;
    constexpr int h = 1 << (t - 1);
    float2 nv[N1W];
    sfor<0, s>([&](auto D) {
      constexpr int d = D;
      sfor<0, h>([&](auto I) {
        constexpr int i = I;
        const float2 a = v[d * 2 * h + i];
        const float2 b = v[d * 2 * h + i + h];
        nv[(d + s) * h + i] = cadd(a, b);
        nv[d * h + i] = twmul_conj<i * s, N1W>(csub(a, b), w1);
      });
    });
    sfor<0, N1W>([&](auto K) { v[K] = nv[K]; });
  });
}

// Non-temporal 8-byte load at byte offset off of a buffer resource; zero past
// its end.
__device__ __forceinline__ float2 load_buf_nt(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  constexpr int kNonTemporal = 2;
  const u2v t = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, kNonTemporal);
  return make_float2(__uint_as_float(t.x), __uint_as_float(t.y));
}

// Rows of dy a wave keeps in flight: four up to n0 = 16, two for n0 = 32,
// whose register rings leave no room for more.
constexpr int adj_prefetch_rows(int n0) { return n0 <= 16 ? 4 : 2; }

// Lanes per column stream of the adjoint (k0 residues). Splitting a stream
// over two lanes halves its rings and its dy registers, so n0 = 32 runs
// without scratch; each load instruction then reads two adjacent k0 rows of
// a window.
constexpr bool adj_kg_built(int n0, int n1, int kg) {
  return kg == 1 || (kg == 2 && n0 >= 8 && n1 <= 32);
}

template <int N0W, int N1W, int KG>
struct AdjCfg {
  static constexpr int M0 = ilog2(N0W);
  static constexpr int G = ilog2(KG);
  static constexpr int QW = 64 / (N1W * KG);                // window columns per strip
  static constexpr int R = 64 / QW;                         // rows per row-adjoint pass
  static constexpr int RING = N0W > 1 ? N0W / 2 : 1;
  static constexpr int PF = adj_prefetch_rows(N0W);         // prefetch depth (rows)
  static constexpr int CR0 = R > RING ? R : RING;
  static constexpr int CR = CR0 > PF ? CR0 : PF;           // rows per chunk
  static constexpr int ZS = N1W + 1;
  static constexpr int ZROW = QW * ZS;
  static constexpr int NL = N0W / KG;                       // dy values per lane and row
  static_assert(KG == 1 || (KG == 2 && N0W >= 4), "streams split over at most two lanes");
  static_assert(N1W * KG <= 64, "one wave holds a whole window column");
  static_assert(CR % PF == 0, "prefetch slots are static");
  static constexpr int WCOLS = QW + N1W - 1;                // x columns a strip touches
};

// Transposed column levels u = m0..1 for one row p (descending order) of a
// stream whose k0 values are split over KG lanes (residue r = lane part):
// on entry g[j] = G_{m0}[p][r + KG j]; the result is G_0[p] = dZ[p] (the same
// in the KG lanes of the stream). ring holds, per level u, the pair sums
// S_u[p'][i] = G_u[p'][i] + G_u[p'][i + h] of the next s_u rows below p
// (already processed) for the nodes i this lane keeps: the layout of ColCfg
// (slot (p mod s_u) * held(u - 1)). For a level whose pairs lie in one lane
// (h = 2^{u-1} >= KG) the pair (i, i + h) has one residue; the level with
// h < KG (u = 1 for KG = 2) combines the two lanes of a stream, whose values
// are exchanged with the partner lane (other(v)). PM = p mod (n0/2), known at
// compile time. conj(Omega0[i s]) = conj(Omega0[r s]) conj(Omega0[KG j s]):
// the lane part comes from lanefac (conj of the forward factor), the uniform
// part from the table; where the uniform part is not 1 or -i, the product
// lwc[u][j] = conj(Omega0[(r + KG j) s]) is precomputed per lane.
template <int N0W, int KG, int PM, typename Other>
__device__ __forceinline__ float2 column_levels_adj(
    const float2 (&g)[N0W / KG], float2 (&ring)[ColCfg<N0W, KG>::RING_TOTAL],
    const float2 (&lanefac)[ColCfg<N0W, KG>::M0 + 1],
    const float2 (&lwc)[ColCfg<N0W, KG>::M0 + 1][ColCfg<N0W, KG>::LW], const float2* w0,
    bool upper, Other&& other) {
  using CC = ColCfg<N0W, KG>;
  float2 cur[N0W / KG];
  sfor<0, N0W / KG>([&](auto K) { cur[K] = g[K]; });
  sfor<0, CC::M0>([&](auto V) {
    constexpr int u = CC::M0 - V;  // M0 .. 1
    constexpr int s = N0W >> u;
    constexpr int hp = CC::held(u - 1);
    constexpr int base = CC::ring_off(u) + (PM % s) * hp;
    if constexpr (u - 1 >= CC::G) {
      // pairs (r + KG j, r + KG j + h) inside the lane: j < hp, partner j + hp
      float2 nxt[N0W / KG];
      sfor<0, hp>([&](auto J) {
        constexpr int j = J;
        const float2 a = cur[j];
        const float2 b = cur[j + hp];
        const float2 below = ring[base + j];
        ring[base + j] = cadd(a, b);
        float2 d = csub(a, b);
        if constexpr (CC::folded(u, j)) {
          d = cmul(lwc[u][j], d);
        } else {
          if constexpr (KG > 1) d = cmul(lanefac[u], d);
          d = twmul_conj<KG * j * s, N0W>(d, w0);
        }
        nxt[j] = cadd(below, d);
      });
      sfor<0, hp>([&](auto K) { cur[K] = nxt[K]; });
    } else {
      // u = 1 with two lanes per stream: the lane of residue 0 holds node 0,
      // its partner node 1; both form node 0 of level 0 (twiddle 1)
      static_assert(u == 1 && KG == 2, "cross-lane level only for KG = 2");
      const float2 mine = cur[0];
      const float2 theirs = other(mine);
      const float2 lo = upper ? theirs : mine;
      const float2 hi = upper ? mine : theirs;
      const float2 below = ring[base];
      ring[base] = cadd(lo, hi);
      cur[0] = cadd(below, csub(lo, hi));
    }
  });
  return cur[0];
}

template <int N0W, int N1W, bool REAL, int KG>
__global__ __launch_bounds__(64) void tree_adj_kernel(const float2* __restrict__ dy,
                                                      void* __restrict__ wsv, AdjGeom g,
                                                      TwiddlesF32 tw) {
  using C = AdjCfg<N0W, N1W, KG>;
  using CC = ColCfg<N0W, KG>;
  __shared__ float2 zl[C::CR * C::ZROW];

  const int lane = threadIdx.x;
  int id = xcd_tile(blockIdx.x, gridDim.x);
  const int strip = id % g.nstrips;
  id /= g.nstrips;
  const int slab = id % g.nslabs;
  const int b = id / g.nslabs;

  const int64_t q1_0 = (int64_t)strip * C::QW;
  const int64_t r0 = (int64_t)slab * g.S;            // first dx row of the slab
  const int64_t r1 = min(r0 + (int64_t)g.S, g.N0);   // one past the last
  // positions run from p_top down to r0; p_top = r1 + n0 - 2 rounded up so
  // that p_top + 1 is a multiple of CR (static ring slots).
  const int64_t p_hi = r1 + N0W - 2;
  const int64_t nsteps_min = p_hi - r0 + 1;
  const int nchunks = (int)((nsteps_min + C::CR - 1) / C::CR);
  const int64_t p_top = r0 + (int64_t)nchunks * C::CR - 1;
  const int64_t q0_last = min(r1 - 1, g.P0 - 1);     // last window row read by this slab

  const float2* dyimg = dy + b * g.y_image_stride;

  // column-phase roles: lane (c, residue, k1)
  const int cp_c = lane / (N1W * KG);
  const int cp_res = (lane / N1W) % KG;
  const int cp_k1 = lane % N1W;
  // dy of one window row of the strip: QW windows from dystrip + q0 *
  // row_bytes, of which the first strip_bytes exist; lanes past the right
  // edge read zero through the buffer resource's range check. A load
  // instruction reads KG adjacent k0 rows of n1 values of each window.
  const float2* dystrip = dyimg + q1_0 * (N0W * N1W);
  const uint64_t row_bytes = (uint64_t)g.P1 * (N0W * N1W * sizeof(float2));
  const uint32_t strip_bytes = uniform_u32(
      (uint32_t)(min((int64_t)C::QW, g.P1 - q1_0) * (N0W * N1W * (int)sizeof(float2))));
  const uint32_t lane_off =
      (uint32_t)((cp_c * (N0W * N1W) + cp_res * N1W + cp_k1) * (int)sizeof(float2));
  // row-phase roles
  const int rp_r = lane / C::QW;
  const int rp_c = lane % C::QW;

  // per-lane twiddle parts of a split stream (see column_levels_adj)
  const float2* const w0 = tw.w0;
  float2 lanefac[CC::M0 + 1];
  float2 lwc[CC::M0 + 1][CC::LW];
  sfor<0, CC::M0 + 1>([&](auto U) {
    constexpr int u = U;
    if constexpr (KG > 1 && u > 0) {
      const float2 f = w0[(cp_res & ((1 << u) - 1)) * (N0W >> u)];
      lanefac[u] = make_float2(f.x, -f.y);
    } else {
      lanefac[u] = make_float2(1.f, 0.f);
    }
    sfor<0, CC::LW>([&](auto J) {
      constexpr int j = J;
      if constexpr (u > 0 && CC::folded(u, j)) {
        const float2 f = w0[((cp_res + KG * j) * (N0W >> u)) % N0W];
        lwc[u][j] = make_float2(f.x, -f.y);
      }
    });
  });
  // the partner lane of a split stream (residue r ^ 1) and which of the two
  // holds node 1 at the cross-lane level
  const bool upper = (cp_res & 1) != 0;
  auto other = [&](float2 v) {
    return make_float2(__shfl_xor(v.x, N1W), __shfl_xor(v.y, N1W));
  };

  float2 ring[CC::RING_TOTAL];
  sfor<0, CC::RING_TOTAL>([&](auto K) { ring[K] = make_float2(0.f, 0.f); });

  // dy rows are loaded in step order gstep = 0, 1, ...: position p = p_top -
  // gstep, window row q0 = p - (n0 - 1). Only q0 in [0, q0_last] with p >= r0
  // exist for this slab (a contiguous range of steps); the others read zeros
  // (an empty resource), which also gives the incomplete trees of Sec. 4.7
  // zero gradient. The row address is a running scalar value.
  const int64_t g_first = p_top - (N0W - 1) - q0_last;
  const int64_t g_last = min(p_top - (N0W - 1), p_top - r0);
  const int64_t g_lo = g_first > 0 ? g_first : 0;
  const StepSpan lsp{(int)uniform_u32((uint32_t)g_lo),
                     uniform_u32((uint32_t)(g_last >= g_lo ? g_last - g_lo + 1 : 0))};
  uint64_t dy_addr = uniform_u64((uint64_t)(uintptr_t)dystrip +
                                 (uint64_t)(p_top - (N0W - 1)) * row_bytes);
  int gstep = 0;
  auto load_step = [&](float2 (&dst)[C::NL]) {
    const auto rs = step_rsrc(dy_addr, gstep, lsp, strip_bytes);
    sfor<0, C::NL>([&](auto K) {
      dst[K] = load_buf_nt(rs, lane_off + K * KG * N1W * (int)sizeof(float2));
    });
    dy_addr -= row_bytes;
    ++gstep;
  };

  float2 pf[C::PF][C::NL];
  sfor<0, C::PF>([&](auto S) { load_step(pf[S]); });

  float* wsr = reinterpret_cast<float*>(wsv);
  float2* wsc = reinterpret_cast<float2*>(wsv);
  const int64_t ws_strip = ((int64_t)b * g.nstrips + strip) * g.N0;  // row base of this strip

  for (int c = 0; c < nchunks; ++c) {
    const int64_t cbase = (int64_t)c * C::CR;
    // chunk rows p = p_top - cbase - st; LDS row st holds dZ[p]
    sfor<0, C::CR>([&](auto STc) {
      constexpr int st = STc;
      constexpr int slot = st % C::PF;
      // p mod (n0/2): p_top + 1 is a multiple of CR, hence of n0/2
      constexpr int pm = (C::RING - 1 - (st % C::RING));
      float2 dz;
      if constexpr (N0W == 1) {
        dz = pf[slot][0];
        load_step(pf[slot]);
      } else if constexpr (N0W / KG >= 32) {
        // the rings fill the registers: use the prefetched row in place and
        // refill its slot afterwards (no second copy of 32 values)
        dz = column_levels_adj<N0W, KG, pm>(pf[slot], ring, lanefac, lwc, tw.w0, upper, other);
        load_step(pf[slot]);
      } else {
        float2 gcur[C::NL];
        sfor<0, C::NL>([&](auto K) { gcur[K] = pf[slot][K]; });
        load_step(pf[slot]);
        dz = column_levels_adj<N0W, KG, pm>(gcur, ring, lanefac, lwc, tw.w0, upper, other);
      }
      // the KG lanes of a stream hold the same dZ; the residue-0 lane writes it
      if (KG == 1 || cp_res == 0) zl[st * C::ZROW + cp_c * C::ZS + cp_k1] = dz;
    });
    __syncthreads();

    // row adjoint for the chunk rows inside [r0, r1), R rows per pass
    sfor<0, C::CR / C::R>([&](auto PS) {
      constexpr int ps = PS;
      const int st = ps * C::R + rp_r;
      float2* zrow = zl + st * C::ZROW + rp_c * C::ZS;
      float2 v[N1W];
      sfor<0, N1W>([&](auto K) { v[K] = zrow[K]; });
      row_levels_adj<N1W>(v, tw.w1);
      // contribution to column q1_0 + rp_c + j is v[n1-1-j]; keep it in place
      // (window columns past the right edge read dy = 0 and contribute 0)
      sfor<0, N1W>([&](auto K) { zrow[K] = v[N1W - 1 - K]; });
      __syncthreads();
      // overlap-add the QW window columns of each row: QW + n1 - 1 partial sums
      for (int o = lane; o < C::R * C::WCOLS; o += 64) {
        const int rr = o / C::WCOLS;
        const int col = o % C::WCOLS;
        const int srow = ps * C::R + rr;
        const int64_t prow = p_top - cbase - srow;
        float2 acc = make_float2(0.f, 0.f);
        const int c_lo = col - (N1W - 1) > 0 ? col - (N1W - 1) : 0;
        const int c_hi = col < C::QW - 1 ? col : C::QW - 1;
        for (int cc = c_lo; cc <= c_hi; ++cc) {
          acc = cadd(acc, zl[srow * C::ZROW + cc * C::ZS + (col - cc)]);
        }
        if (prow >= r0 && prow < r1) {
          const int64_t idx = (ws_strip + prow) * C::WCOLS + col;
          if constexpr (REAL) {
            wsr[idx] = acc.x * g.scale;
          } else {
            wsc[idx] = make_float2(acc.x * g.scale, acc.y * g.scale);
          }
        }
      }
      __syncthreads();
    });
  }
}

// dx[b][r][c] = sum over strips s whose columns [s*QW, s*QW + QW + n1 - 1)
// contain c of ws[b][s][r][c - s*QW], in ascending s. One workgroup per
// (block of kAdjReduceRows image rows, block of kAdjReduceThreads columns):
// the rows come from the workgroup index (scalar arithmetic), each lane takes
// one column of each of the rows and issues the loads of all of them before
// it adds (one row per lane measured 14.2 -> 11.5 us at 16 x 256^2, the
// loads of several rows at once less again).
constexpr int kAdjReduceThreads = 256;
constexpr int kAdjReduceRows = 4;

template <int QW, int N1W, bool REAL>
__global__ __launch_bounds__(kAdjReduceThreads) void tree_adj_reduce_kernel(
    const void* __restrict__ wsv, void* __restrict__ dxv, AdjGeom g, int cblocks) {
  constexpr int WCOLS = QW + N1W - 1;
  constexpr int RR = kAdjReduceRows;
  const int rblock = (int)blockIdx.x / cblocks;       // rows rblock * RR .. + RR of b * N0 + r
  const int cb = (int)blockIdx.x - rblock * cblocks;
  const int64_t c = (int64_t)cb * kAdjReduceThreads + threadIdx.x;
  if (c >= g.N1) return;
  const int nrows = g.batch * (int)g.N0;
  int64_t s_lo = c - (WCOLS - 1);
  s_lo = s_lo > 0 ? (s_lo + QW - 1) / QW : 0;
  int64_t s_hi = c / QW;
  if (s_hi > g.nstrips - 1) s_hi = g.nstrips - 1;
  // ws index of (b, s, r, c - s*QW): base + s * (N0 * WCOLS - QW). At most
  // NS strips cover a column; the loads past s_hi (and of rows past the
  // last) read an in-range element and are not added.
  constexpr int NS = (WCOLS + QW - 1) / QW;
  const int64_t step = g.N0 * WCOLS - QW;
  const int cnt = (int)(s_hi - s_lo + 1);
  using T = std::conditional_t<REAL, float, float2>;
  const T* ws = reinterpret_cast<const T*>(wsv);
  T part[RR][NS];
  int64_t out[RR];
  sfor<0, RR>([&](auto KR) {
    constexpr int kr = KR;
    const int row0 = rblock * RR + kr;
    const int row = row0 < nrows ? row0 : nrows - 1;
    const int b = row / (int)g.N0;
    const int r = row - b * (int)g.N0;
    out[kr] = row0 < nrows ? (int64_t)row * g.N1 + c : -1;
    const int64_t idx0 =
        (((int64_t)b * g.nstrips + s_lo) * g.N0 + r) * WCOLS + (c - s_lo * QW);
    sfor<0, NS>([&](auto K) {
      constexpr int k = K;
      part[kr][k] = ws[idx0 + (k < cnt ? k : 0) * step];
    });
  });
  sfor<0, RR>([&](auto KR) {
    constexpr int kr = KR;
    T acc = part[kr][0];
    sfor<1, NS>([&](auto K) {
      constexpr int k = K;
      if constexpr (REAL) {
        acc += k < cnt ? part[kr][k] : 0.f;
      } else {
        acc = cadd(acc, k < cnt ? part[kr][k] : make_float2(0.f, 0.f));
      }
    });
    if (out[kr] >= 0) reinterpret_cast<T*>(dxv)[out[kr]] = acc;
  });
}

template <int N0W, int N1W, bool REAL, int KG>
hipError_t launch_adj_kg(const float2* dy, void* ws, void* dx, const AdjGeom& g,
                         const TwiddlesF32& tw, hipStream_t stream) {
  const int64_t nb = (int64_t)g.batch * g.nslabs * g.nstrips;
  using C = AdjCfg<N0W, N1W, KG>;
  const unsigned pad =
      occupancy_lds(g.wpc, g.lds_cu, C::CR * C::ZROW * (unsigned)sizeof(float2));
  hipLaunchKernelGGL((tree_adj_kernel<N0W, N1W, REAL, KG>), dim3((unsigned)nb), dim3(64), pad,
                     stream, dy, ws, g, tw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int cblocks = (int)((g.N1 + kAdjReduceThreads - 1) / kAdjReduceThreads);
  const int64_t rblocks = ((int64_t)g.batch * g.N0 + kAdjReduceRows - 1) / kAdjReduceRows;
  hipLaunchKernelGGL((tree_adj_reduce_kernel<C::QW, N1W, REAL>),
                     dim3((unsigned)(rblocks * cblocks)), dim3(kAdjReduceThreads), 0, stream, ws,
                     dx, g, cblocks);
  return hipGetLastError();
}

template <int N0W, int N1W, bool REAL>
hipError_t launch_adj_one(const float2* dy, void* ws, void* dx, const AdjGeom& g,
                          const TwiddlesF32& tw, hipStream_t stream) {
  if constexpr (adj_kg_built(N0W, N1W, 2)) {
    if (g.kg == 2) return launch_adj_kg<N0W, N1W, REAL, 2>(dy, ws, dx, g, tw, stream);
  }
  if (g.kg == 1) return launch_adj_kg<N0W, N1W, REAL, 1>(dy, ws, dx, g, tw, stream);
  return hipErrorInvalidValue;
}

template <int N0W, bool REAL>
hipError_t launch_adj_n0(int n1, const float2* dy, void* ws, void* dx, const AdjGeom& g,
                         const TwiddlesF32& tw, hipStream_t s) {
  switch (n1) {
    case 1: return launch_adj_one<N0W, 1, REAL>(dy, ws, dx, g, tw, s);
    case 2: return launch_adj_one<N0W, 2, REAL>(dy, ws, dx, g, tw, s);
    case 4: return launch_adj_one<N0W, 4, REAL>(dy, ws, dx, g, tw, s);
    case 8: return launch_adj_one<N0W, 8, REAL>(dy, ws, dx, g, tw, s);
    case 16: return launch_adj_one<N0W, 16, REAL>(dy, ws, dx, g, tw, s);
    case 32: return launch_adj_one<N0W, 32, REAL>(dy, ws, dx, g, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tree

#define SWDFT_ADJ_DECL(N0W, TAG) \
  hipError_t launch_tree_adj_n0_##N0W##_##TAG(int, const float2*, void*, void*, const AdjGeom&, \
                                             const TwiddlesF32&, hipStream_t);
SWDFT_ADJ_DECL(1, r)
SWDFT_ADJ_DECL(1, c)
SWDFT_ADJ_DECL(2, r)
SWDFT_ADJ_DECL(2, c)
SWDFT_ADJ_DECL(4, r)
SWDFT_ADJ_DECL(4, c)
SWDFT_ADJ_DECL(8, r)
SWDFT_ADJ_DECL(8, c)
SWDFT_ADJ_DECL(16, r)
SWDFT_ADJ_DECL(16, c)
SWDFT_ADJ_DECL(32, r)
SWDFT_ADJ_DECL(32, c)
#undef SWDFT_ADJ_DECL

}  // namespace swdft
