// Mixed-radix fused forward 2D Tree SWDFT for gfx950: window sides of the
// form 2^a 3^b. The tree of Sec. 4.2 is binary because the FFT it follows is
// radix-2; a radix-3 factor turns a level into ternary trees (Sec. 5), and a
// side such as 12 = 2 * 2 * 3 mixes both.
//
// Levels. A side n = r_1 r_2 ... r_m is factored with the twos first, then
// the threes. Level t has L_t = r_1 ... r_t values per node and shift
// s_t = n / L_t: the node of level t at position p is the L_t-point DFT of the
// samples p - (L_t - 1) s_t, ..., p - s_t, p. It combines the r = r_t nodes of
// level t-1 at positions p - (r - 1 - j) s_t, j < r (the j-th decimated
// subsequence of those samples):
//   a_j = Omega[i j s_t] T_{t-1}[p - (r - 1 - j) s_t][i],        i < L_{t-1}
//   T_t[p][i + q L_{t-1}] = sum_{j<r} w_r^{q j} a_j,            q < r,
// with w_r = Omega[n / r]. For r = 2 this is Eq. (5) (rows) and Eq. (6)
// (columns); for r = 3 the butterfly is the 3-point DFT
//   X0 = a0 + (a1 + a2),  X1,2 = a0 - (a1 + a2) / 2 -/+ i (sqrt(3)/2) (a1 - a2).
// The last level holds the n bins in natural order.
//
// Mapping (as the radix-2 kernel with unsplit streams and one wave per strip):
//  * QW = floor(64 / n1) window columns per wave; lane (c, k1) of the column
//    phase owns stream (q1_0 + c, k1), lanes past QW n1 idle (their stores
//    fall outside the buffer resource).
//  * Row phase: lane (r, c) computes the row levels for one position from
//    its n1 inputs (neighbours recomputed), R = floor(64 / QW) rows per pass,
//    into LDS.
//  * Column phase: level u keeps level-(u-1) nodes of the last (r_u - 1) s_u
//    positions in a register ring, slot p mod ((r_u - 1) s_u). Chunks of CR
//    rows start at multiples of the least common multiple of the ring
//    lengths (the period), and one period is unrolled, so every slot is a
//    fixed register; a loop repeats it over the chunk. Each
//    new row costs one new tree column: per level u, (r_u - 1) L_{u-1}
//    twiddle products and L_{u-1} butterflies of r_u points.
//  * Output: plain stores except for n1 = 16, where a store covers whole
//    128-byte lines of a window; inputs of the next chunk are loaded before
//    the column phase of the current one. Resident workgroups per CU may be
//    capped and tiles then run in dispatch order, as for the radix-2 kernel.
#pragma once

#include "tree_fwd_kernel.h"

namespace swdft {
namespace mixed {

using tree::buf_rsrc;
using tree::cadd;
using tree::cmul;
using tree::csub;
using tree::kOutOfRange;
using tree::load_buf;
using tree::sfor;
using tree::store_buf;
using tree::uload;
using tree::uniform_copy;
using tree::xcd_tile;

constexpr bool radix23(int n) {
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}
constexpr int twos(int n) { return n % 2 == 0 ? 1 + twos(n / 2) : 0; }
constexpr int threes(int n) { return n % 3 == 0 ? 1 + threes(n / 3) : 0; }
constexpr int gcd(int a, int b) { return b == 0 ? a : gcd(b, a % b); }
constexpr int lcm(int a, int b) { return a / gcd(a, b) * b; }

// The factorisation of one side: radix of level t (1-based), values per node
// L_t and shift s_t.
template <int N>
struct Radix {
  static_assert(radix23(N), "window side must be 2^a 3^b");
  static constexpr int A = twos(N);
  static constexpr int M = A + threes(N);  // number of levels
  static constexpr int r(int t) { return t <= A ? 2 : 3; }
  static constexpr int L(int t) { return t == 0 ? 1 : L(t - 1) * r(t); }
  static constexpr int s(int t) { return N / L(t); }
  // ring of level t: level-(t-1) nodes of the last (r_t - 1) s_t positions
  static constexpr int ring_len(int t) { return (r(t) - 1) * s(t); }
  static constexpr int ring_size(int t) { return ring_len(t) * L(t - 1); }
  static constexpr int ring_off(int t) { return t <= 1 ? 0 : ring_off(t - 1) + ring_size(t - 1); }
  static constexpr int RING_TOTAL = M > 0 ? ring_off(M + 1) : 1;
  static constexpr int period(int t = 1) {
    return t > M ? 1 : lcm(ring_len(t), period(t + 1));
  }
};

// d * Omega[IDX] for a length-N twiddle vector, IDX < N known at compile
// time; quarter and half turns are exact.
template <int IDX, int N>
__device__ __forceinline__ float2 twmul_any(float2 d, const float2* w) {
  if constexpr (IDX == 0) {
    return d;
  } else if constexpr (4 * IDX == N) {
    return make_float2(d.y, -d.x);
  } else if constexpr (2 * IDX == N) {
    return make_float2(-d.x, -d.y);
  } else if constexpr (4 * IDX == 3 * N) {
    return make_float2(-d.y, d.x);
  } else {
    return cmul(uload(w + IDX), d);
  }
}

// The r-point butterfly of a level on the twiddled inputs a[0..r): out(q, X_q).
template <int RADIX, int N, typename Out>
__device__ __forceinline__ void butterfly(const float2 (&a)[3], const float2* w, Out&& out) {
  if constexpr (RADIX == 2) {
    out(std::integral_constant<int, 0>{}, cadd(a[0], a[1]));
    out(std::integral_constant<int, 1>{}, csub(a[0], a[1]));
  } else {
    // sqrt(3)/2 = -Im Omega[N/3], from the FP64-generated table. Every
    // rounding is written out (fused multiply-adds): X1,2 = t2 -/+ i c3 d
    // with t2 = a0 - t1 / 2.
    const float c3 = -uload(w + N / 3).y;
    const float2 t1 = cadd(a[1], a[2]);
    const float2 t2 = make_float2(__builtin_fmaf(-0.5f, t1.x, a[0].x),
                                  __builtin_fmaf(-0.5f, t1.y, a[0].y));
    const float2 d = csub(a[1], a[2]);
    out(std::integral_constant<int, 0>{}, cadd(a[0], t1));
    out(std::integral_constant<int, 1>{}, make_float2(__builtin_fmaf(c3, d.y, t2.x),
                                                      __builtin_fmaf(-c3, d.x, t2.y)));
    out(std::integral_constant<int, 2>{}, make_float2(__builtin_fmaf(-c3, d.y, t2.x),
                                                      __builtin_fmaf(c3, d.x, t2.y)));
  }
}

// Row levels for one position p from v[d] = x[p - d], d < n1. Level t holds,
// for offsets d < s_t, the L_t values of the node at p - d at [d L_t + i].
template <int N1W>
__device__ __forceinline__ void row_levels(float2 (&v)[N1W], const float2* w1) {
  using RX = Radix<N1W>;
  sfor<1, RX::M + 1>([&](auto T) {
    constexpr int t = T;
    constexpr int r = RX::r(t);
    constexpr int s = RX::s(t);
    constexpr int lp = RX::L(t - 1);
    float2 nv[N1W];
    sfor<0, s>([&](auto D) {
      constexpr int d = D;
      sfor<0, lp>([&](auto I) {
        constexpr int i = I;
        float2 a[3];
        sfor<0, r>([&](auto J) {
          constexpr int j = J;
          a[j] = twmul_any<i * j * s, N1W>(v[(d + (r - 1 - j) * s) * lp + i], w1);
        });
        butterfly<r, N1W>(a, w1, [&](auto Q, float2 x) { nv[d * lp * r + i + Q * lp] = x; });
      });
    });
    sfor<0, N1W>([&](auto K) { v[K] = nv[K]; });
  });
}

// Column levels for one new row (step ST of a chunk that starts at a multiple
// of the ring period): z is level 0 of the new position. emit(k0, value).
// T0 >= 0 marks the row as the T0-th of a slab whose first window starts at
// the slab's first row: level u of the row feeds only the windows ending at
// rows p .. p + s_u - 1, so below T0 = n0 - 1 it is computed only when
// T0 >= n0 - s_u, and level u-1 is kept in the ring only when
// T0 >= n0 - s_{u-1} (its last reader, level u at p + (r_u - 1) s_u, is then
// used). T0 = -1 computes every level.
template <int N0W, int ST, int T0 = -1, typename Emit>
__device__ __forceinline__ void column_levels(float2 z, float2 (&ring)[Radix<N0W>::RING_TOTAL],
                                              const float2* w0, Emit&& emit) {
  using RX = Radix<N0W>;
  float2 cur[N0W];
  cur[0] = z;
  sfor<1, RX::M + 1>([&](auto U) {
    constexpr int u = U;
    constexpr int r = RX::r(u);
    constexpr int s = RX::s(u);
    constexpr int lp = RX::L(u - 1);
    constexpr int len = RX::ring_len(u);
    constexpr int off = RX::ring_off(u);
    constexpr bool level_in = T0 < 0 || T0 >= N0W - RX::s(u - 1);  // level u-1 used
    constexpr bool level_out = T0 < 0 || T0 >= N0W - s;            // level u used
    if constexpr (!level_in) {
      // nothing of this level or above is used at this row
    } else if constexpr (!level_out) {
      sfor<0, lp>([&](auto I) { ring[off + (ST % len) * lp + I] = cur[I]; });
    } else {
    float2 nxt[N0W];
    sfor<0, lp>([&](auto I) {
      constexpr int i = I;
      float2 a[3];
      // subsequence j < r - 1 is the node of position p - (r - 1 - j) s
      sfor<0, r - 1>([&](auto J) {
        constexpr int j = J;
        constexpr int slot = ((ST - (r - 1 - j) * s) % len + len) % len;
        a[j] = twmul_any<i * j * s, N0W>(ring[off + slot * lp + i], w0);
      });
      a[r - 1] = twmul_any<i * (r - 1) * s, N0W>(cur[i], w0);
      butterfly<r, N0W>(a, w0, [&](auto Q, float2 x) {
        if constexpr (u == RX::M) {
          emit(std::integral_constant<int, i + Q * lp>{}, x);
        } else {
          nxt[i + Q * lp] = x;
        }
      });
    });
    // position p takes the slot of p - (r - 1) s, read above
    sfor<0, lp>([&](auto I) { ring[off + (ST % len) * lp + I] = cur[I]; });
    if constexpr (u < RX::M) {
      sfor<0, lp * r>([&](auto K) { cur[K] = nxt[K]; });
    }
    }
  });
}

// Period of the column rings of side n0 (least common multiple of their
// lengths), computed without the templates for the host.
constexpr int ring_period(int n0) {
  int a = twos(n0), b = threes(n0), L = 1, period = 1;
  for (int t = 1; t <= a + b; ++t) {
    const int rad = t <= a ? 2 : 3;
    L *= rad;
    period = lcm(period, (rad - 1) * (n0 / L));
  }
  return period;
}

// Rows per chunk: a common multiple of the rows of one row pass and of the
// ring period, at least 16.
constexpr int rows_per_chunk(int n0, int n1) {
  const int r = 64 / (64 / n1);
  const int base = lcm(r, ring_period(n0));
  return base >= 16 ? base : base * ((16 + base - 1) / base);
}

template <int N0W, int N1W, bool REAL>
struct MixedCfg {
  static constexpr int QW = 64 / N1W;                       // window columns per strip
  static constexpr int R = 64 / QW;                         // rows per row pass
  static constexpr int PERIOD = Radix<N0W>::period();
  static_assert(PERIOD == ring_period(N0W), "ring period");
  static constexpr int CR = rows_per_chunk(N0W, N1W);
  static constexpr int PPW = CR / R;                        // row passes per chunk
  static constexpr int ZS = N1W + 1;
  static constexpr int ZROW = QW * ZS;
  static constexpr int LDS_FLOAT2 = CR * ZROW;
  static constexpr bool NT_STORES = N1W == 16;
  static_assert((int64_t)CR * SWDFT_MAX_ROW * 8 <= (int64_t)kOutOfRange,
                "one chunk of input rows must stay addressable with 32-bit offsets");
};

template <int N0W, int N1W, bool REAL>
__global__ __launch_bounds__(64) void tree_mixed_kernel(const void* __restrict__ xv,
                                                        float2* __restrict__ y, TreeGeom g_in,
                                                        TwiddlesF32 tw) {
  using C = MixedCfg<N0W, N1W, REAL>;
  __shared__ float2 zl[C::LDS_FLOAT2];
  const TreeGeom g = uniform_copy(g_in);
  int id = g.order ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
  const int strip = id % g.nstrips;
  id /= g.nstrips;
  const int slab = id % g.nslabs;
  const int b = id / g.nslabs;
  const int lane = threadIdx.x;
  const float2* w0 = tw.w0;
  const float2* w1 = tw.w1;

  const int64_t q1_0 = (int64_t)strip * C::QW;
  const int64_t row0 = (int64_t)slab * g.S;
  const int64_t q0_end = min(row0 + (int64_t)g.S, g.P0);
  const int nrows = (int)(q0_end - row0) + N0W - 1;
  const int nchunks = (nrows + C::CR - 1) / C::CR;

  using XT = std::conditional_t<REAL, float, float2>;
  constexpr int EB = (int)sizeof(XT);
  const XT* ximg = reinterpret_cast<const XT*>(xv) + b * g.x_image_stride;
  float2* yimg = y + b * g.y_image_stride;

  // row-phase roles: lane (r, c); lanes past R * QW idle
  const int rp_r = lane / C::QW;
  const int rp_c = lane % C::QW;
  const bool rp_live = rp_r < C::R;
  const int64_t rp_q1 = q1_0 + rp_c;
  uint32_t x_off[N1W];
  sfor<0, N1W>([&](auto D) {
    constexpr int d = D;
    const int64_t col = rp_q1 + (N1W - 1 - d);
    x_off[d] = (rp_live && col < g.N1) ? (uint32_t)(((int64_t)rp_r * g.N1 + col) * EB)
                                       : kOutOfRange;
  });
  XT xin[C::PPW][N1W];
  auto load_chunk = [&](int64_t crow) __attribute__((always_inline)) {
    // scalar values, so that the loads need no loop over distinct
    // resources (the device min template goes through double precision)
    const int64_t rows = tree::clamp_i64(g.N0 - crow, 0, C::CR);
    const auto rs = buf_rsrc(
        (const void*)(uintptr_t)tree::uniform_u64((uint64_t)(uintptr_t)(ximg + (rows > 0 ? crow : 0) * g.N1)),
        tree::uniform_u32((uint32_t)(rows * g.N1 * EB)));
    sfor<0, C::PPW>([&](auto PS) {
      constexpr int ps = PS;
      sfor<0, N1W>([&](auto D) {
        constexpr int d = D;
        xin[ps][d] = load_buf<REAL>(rs, x_off[d] + (uint32_t)(ps * C::R * g.N1 * EB));
      });
    });
  };

  // column-phase roles: lane (c, k1); lanes past QW n1 idle
  const int cp_c_raw = lane / N1W;
  const bool cp_live = cp_c_raw < C::QW;
  const int cp_c = cp_live ? cp_c_raw : C::QW - 1;
  const int cp_k1 = lane % N1W;
  float2* ystrip = yimg + q1_0 * (N0W * N1W);
  const uint64_t row_bytes = (uint64_t)g.P1 * (N0W * N1W * sizeof(float2));
  const uint32_t strip_bytes = tree::uniform_u32(
      (uint32_t)(min((int64_t)C::QW, g.P1 - q1_0) * (N0W * N1W * (int)sizeof(float2))));
  const uint32_t lane_off =
      cp_live ? (uint32_t)((cp_c * (N0W * N1W) + cp_k1) * (int)sizeof(float2)) : kOutOfRange;

  float2 ring[Radix<N0W>::RING_TOTAL];
  sfor<0, Radix<N0W>::RING_TOTAL>([&](auto K) { ring[K] = make_float2(0.f, 0.f); });

  auto row_phase = [&]() __attribute__((always_inline)) {
    sfor<0, C::PPW>([&](auto PS) {
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
      if (g.scale != 1.0f) {
        sfor<0, N1W>([&](auto K) { v[K] = make_float2(v[K].x * g.scale, v[K].y * g.scale); });
      }
      if (rp_live) {
        float2* zrow = zl + (ps * C::R + rp_r) * C::ZROW + rp_c * C::ZS;
        sfor<0, N1W>([&](auto K) { zrow[K] = v[K]; });
      }
    });
  };

  load_chunk(row0);
  row_phase();
  __syncthreads();
  for (int c = 0; c < nchunks; ++c) {
    const int64_t crow = row0 + (int64_t)c * C::CR;
    if (c + 1 < nchunks) load_chunk(crow + C::CR);
    __builtin_amdgcn_sched_barrier(0);
    // one ring period unrolled (its slots are fixed registers), repeated
    const float2* zcol = zl + cp_c * C::ZS + cp_k1;
    // step `row` writes window row q0 = crow + row - (n0 - 1) if it lies in the slab
    const tree::StepSpan sp = tree::step_span(crow, row0, q0_end, N0W - 1, C::CR);
    uint64_t row_addr = tree::uniform_u64((uint64_t)(uintptr_t)ystrip +
                                          (uint64_t)(crow - (N0W - 1)) * row_bytes);
    // step `row` of period sc; T0 >= 0 (the slab's first chunk, whose row
    // `row` is the slab's row `row`) lets the priming steps skip the levels
    // no window of the slab uses
    auto period = [&](int sc, auto T0BASE) __attribute__((always_inline)) {
      sfor<0, C::PERIOD>([&](auto STc) {
        constexpr int st = STc;
        const int row = sc * C::PERIOD + st;
        const float2 z = zcol[row * C::ZROW];
        const auto out = tree::step_rsrc(row_addr, row, sp, strip_bytes);
        row_addr += row_bytes;
        if constexpr (N0W == 1) {
          store_buf<C::NT_STORES>(out, lane_off, z);
        } else {
          constexpr int t0 = T0BASE < 0 ? -1 : T0BASE + st;
          column_levels<N0W, st, t0>(z, ring, w0, [&](auto K, float2 v) {
            store_buf<C::NT_STORES>(out, lane_off + K * N1W * (int)sizeof(float2), v);
          });
        }
      });
    };
    // the first periods of the slab's first chunk, which hold its priming
    // steps, are unrolled once more with their row index known
    constexpr int kPrimePeriods0 = (N0W - 1 + C::PERIOD - 1) / C::PERIOD;
    constexpr int kPrimePeriods =
        kPrimePeriods0 < C::CR / C::PERIOD ? kPrimePeriods0 : C::CR / C::PERIOD;
    int sc0 = 0;
    if (c == 0) {
      sfor<0, kPrimePeriods>([&](auto SC) {
        period(SC, std::integral_constant<int, SC * C::PERIOD>{});
      });
      sc0 = kPrimePeriods;
    }
#pragma clang loop unroll(disable)
    for (int sc = sc0; sc < C::CR / C::PERIOD; ++sc) period(sc, std::integral_constant<int, -1>{});
    __syncthreads();
    if (c + 1 < nchunks) {
      row_phase();
      __syncthreads();
    }
  }
}

template <int N0W, int N1W, bool REAL>
hipError_t launch_one(const void* x, float2* y, const TreeGeom& g, const TwiddlesF32& tw,
                      hipStream_t stream) {
  const int64_t nb = (int64_t)g.batch * g.nslabs * g.nstrips;
  if (nb < 1 || nb > 0x7fffffff) return hipErrorInvalidConfiguration;
  // optional cap on resident workgroups per CU, as for the radix-2 kernel
  const unsigned pad = tree::occupancy_lds(
      g.wpc, g.lds_cu, MixedCfg<N0W, N1W, REAL>::LDS_FLOAT2 * (unsigned)sizeof(float2));
  hipLaunchKernelGGL((tree_mixed_kernel<N0W, N1W, REAL>), dim3((unsigned)nb), dim3(64), pad,
                     stream, x, y, g, tw);
  return hipGetLastError();
}

// Sides of the mixed-radix kernels: 3, 6, 9, 12, 24 with each other and with
// 4, 8, 16 (pure powers of two run the radix-2 kernels).
#define SWDFT_MIXED_N1_CASES(N0W, REAL)                                        \
  case 3: return launch_one<N0W, 3, REAL>(x, y, g, tw, s);                     \
  case 4: return launch_one<N0W, 4, REAL>(x, y, g, tw, s);                     \
  case 6: return launch_one<N0W, 6, REAL>(x, y, g, tw, s);                     \
  case 8: return launch_one<N0W, 8, REAL>(x, y, g, tw, s);                     \
  case 9: return launch_one<N0W, 9, REAL>(x, y, g, tw, s);                     \
  case 12: return launch_one<N0W, 12, REAL>(x, y, g, tw, s);                   \
  case 16: return launch_one<N0W, 16, REAL>(x, y, g, tw, s);                   \
  case 24: return launch_one<N0W, 24, REAL>(x, y, g, tw, s);

#define SWDFT_MIXED_N1_CASES_ODD(N0W, REAL)                                    \
  case 3: return launch_one<N0W, 3, REAL>(x, y, g, tw, s);                     \
  case 6: return launch_one<N0W, 6, REAL>(x, y, g, tw, s);                     \
  case 9: return launch_one<N0W, 9, REAL>(x, y, g, tw, s);                     \
  case 12: return launch_one<N0W, 12, REAL>(x, y, g, tw, s);                   \
  case 24: return launch_one<N0W, 24, REAL>(x, y, g, tw, s);

// n1 launchers for one n0: every side for a mixed n0, the mixed sides for a
// power-of-two n0.
template <int N0W, bool REAL>
hipError_t launch_n0(int n1, const void* x, float2* y, const TreeGeom& g, const TwiddlesF32& tw,
                     hipStream_t s) {
  if constexpr ((N0W & (N0W - 1)) != 0) {
    switch (n1) {
      SWDFT_MIXED_N1_CASES(N0W, REAL)
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (n1) {
      SWDFT_MIXED_N1_CASES_ODD(N0W, REAL)
      default: return hipErrorInvalidValue;
    }
  }
}

}  // namespace mixed

hipError_t launch_tree_mixed_r(int n0, int n1, const void* x, float2* y, const TreeGeom& g,
                               const TwiddlesF32& tw, hipStream_t s);
hipError_t launch_tree_mixed_c(int n0, int n1, const void* x, float2* y, const TreeGeom& g,
                               const TwiddlesF32& tw, hipStream_t s);

}  // namespace swdft
