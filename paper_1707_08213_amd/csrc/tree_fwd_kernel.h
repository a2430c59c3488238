// Fused forward 2D Tree SWDFT for gfx950.
//
// The tree of Sec. 4.2 is a row-column radix-2 decimation-in-time FFT whose
// nodes are indexed by window position. Row levels t = 1..m1 (Eq. (5)) build,
// for every position p1, the n1-point DFT Z[p0][q1][k1] of the row segment
// x[p0][q1 .. q1+n1-1]; column levels v = m1+1..m1+m0 (Eq. (6)) then build the
// n0-point DFT of each column of Z, which is the 2D DFT of the window. The
// final level is the output (Sec. 4.2, last paragraph).
//
// Mapping to the hardware (one wave64 per workgroup, waves independent):
//  * A wave owns QW = 64/n1 adjacent window columns and a slab of S output
//    rows of one image. Lane (c, k1) of the column phase owns the stream
//    Z[.][q1_0 + c][k1] and walks it down the slab one input row per step.
//  * Column phase (Eq. (6)), in registers: at row p a lane needs level u-1 of
//    its own tree (p) and of tree p - s_u, s_u = n0 / 2^u. It keeps the last
//    s_u positions of every level u-1 in a register ring (n0/2 complex values
//    per level, m0 levels). Rows are processed in chunks whose length is a
//    multiple of the ring period n0/2, and each chunk is fully unrolled, so
//    every ring slot is a fixed register. Each new row costs the
//    2 + 4 + ... + n0 = 2(n0-1) node operations of one new tree column
//    (Eq. (8)); the last level is written straight from registers.
//  * Row phase (Eq. (5)), once per chunk: lane (r, c) takes input row r of
//    the chunk and window column c, runs the m1 row levels for that tree
//    position (the nodes of the neighbouring positions it depends on are
//    recomputed by this lane) and leaves the n1 row DFTs in LDS. Z never
//    reaches HBM.
//  * Output: for each k0 the 64 lanes store QW full n1*8-byte rows of
//    consecutive windows, i.e. whole 128-byte lines, with non-temporal
//    stores; the output is the only large HBM stream.
//  * The first n0-1 rows of a slab only prime the rings (their windows belong
//    to the previous slab); their outputs are not stored. Partial trees near
//    the top and left edges (Sec. 4.7) read zeros and are never stored.
//  * Workgroup ids are remapped so that each XCD (own L2) gets a contiguous
//    range of tiles: neighbouring strips share input columns.
#pragma once
#include <type_traits>

#include "internal.h"

namespace swdft {
namespace tree {

typedef float f2v __attribute__((ext_vector_type(2)));

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// Load a value that is the same for every lane of the wave and keep it in
// scalar registers. Used for twiddles and tile geometry, which the persistent
// batched kernel reads from a device table at addresses the compiler cannot
// prove unmodified (so it would otherwise hold them in vector registers).
__device__ __forceinline__ float2 uload(const float2* p) {
  const float2 v = *p;
  return make_float2(__builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v.x))),
                     __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v.y))));
}

template <typename T>
__device__ __forceinline__ T uniform_copy(const T& src) {
  static_assert(sizeof(T) % 4 == 0, "dword-sized");
  struct Words { int w[sizeof(T) / 4]; };
  const Words in = __builtin_bit_cast(Words, src);
  Words out;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) out.w[i] = __builtin_amdgcn_readfirstlane(in.w[i]);
  return __builtin_bit_cast(T, out);
}

// d * Omega[IDX] for a length-N twiddle vector, IDX < N/2 known at compile
// time. Omega[0] = 1 and Omega[N/4] = -i are applied exactly without a
// multiply; every other value comes from the FP64-generated table.
template <int IDX, int N>
__device__ __forceinline__ float2 twmul(float2 d, const float2* w) {
  if constexpr (IDX == 0) {
    return d;
  } else if constexpr (4 * IDX == N) {
    return make_float2(d.y, -d.x);
  } else {
    const float2 t = uload(w + IDX);
    return make_float2(t.x * d.x - t.y * d.y, t.x * d.y + t.y * d.x);
  }
}

// Row levels t = 1..m1 (Eq. (5)) for the single tree position p whose
// level-0 neighbours are v[d] = x[p - d], d < n1. Level t holds, for offsets
// d < s_t = n1 / 2^t, the nodes i < 2^t at [d * 2^t + i]:
//   T_t[d][i]     = T_{t-1}[d + s_t][i] + Omega1[i s_t] T_{t-1}[d][i]
//   T_t[d][i + h] = T_{t-1}[d + s_t][i] - Omega1[i s_t] T_{t-1}[d][i]
// (h = 2^{t-1}; Omega1[(i + h) s_t] = -Omega1[i s_t]). On return v[k1] is the
// n1-point DFT of x[p-n1+1 .. p] at bin k1, in natural order.
template <int N1W>
__device__ __forceinline__ void row_levels(float2 (&v)[N1W], const float2* w1) {
  constexpr int M1 = ilog2(N1W);
  sfor<1, M1 + 1>([&](auto T) {
    constexpr int t = T;
    constexpr int s = N1W >> t;
    constexpr int h = 1 << (t - 1);
    float2 nv[N1W];
    sfor<0, s>([&](auto D) {
      constexpr int d = D;
      sfor<0, h>([&](auto I) {
        constexpr int i = I;
        const float2 b = v[(d + s) * h + i];
        const float2 tw = twmul<i * s, N1W>(v[d * h + i], w1);
        nv[d * 2 * h + i] = cadd(b, tw);
        nv[d * 2 * h + i + h] = csub(b, tw);
      });
    });
    sfor<0, N1W>([&](auto K) { v[K] = nv[K]; });
  });
}

// Column phase bookkeeping for a stream split over KG lanes (KG = 2^G, a
// power of two below n0). Lane residue r < KG holds, at level v, the nodes
// i < 2^v with i = r (mod KG): one node (i = r mod 2^v) while 2^v <= KG, else
// the 2^v / KG nodes r + KG j. Those nodes depend only on level-(v-1) nodes
// of the same residue, so the KG lanes never exchange data; the k0 outputs
// of lane r are k0 = r + KG j.
template <int N0W, int KG>
struct ColCfg {
  static constexpr int M0 = ilog2(N0W);
  static constexpr int G = ilog2(KG);
  static constexpr int held(int v) { return v <= G ? 1 : (1 << v) / KG; }
  // the ring read at level u holds level u-1 of the last s_u = n0/2^u trees
  static constexpr int ring_size(int u) { return (N0W >> u) * held(u - 1); }
  static constexpr int ring_off(int u) { return u <= 1 ? 0 : ring_off(u - 1) + ring_size(u - 1); }
  static constexpr int RING_TOTAL = M0 > 0 ? ring_off(M0 + 1) : 1;
  static constexpr int OUTS = N0W / KG;  // outputs per lane and row
};

// Column levels u = 1..m0 (Eq. (6)) for one new row p of a (q1, k1) stream:
//   T_u[p][i]     = T_{u-1}[p - s_u][i] + Omega0[i s_u] T_{u-1}[p][i]
//   T_u[p][i + h] = T_{u-1}[p - s_u][i] - Omega0[i s_u] T_{u-1}[p][i]
// The ring of level u-1 keeps its last s_u trees, slot (p mod s_u); the slot
// read for tree p - s_u is the slot tree p is written to. ST is the row index
// within the chunk (chunks start at multiples of n0/2, so p mod s_u = ST mod s_u).
// For a split stream (KG > 1) the twiddle of node r + KG j is
// Omega0[(r + KG j) s_u] = lanefac[u] * Omega0[KG j s_u]: a per-lane factor
// (lanefac[u] = Omega0[(r mod 2^u) s_u]) times a twiddle uniform over the wave.
// emit(j, v) receives output k0 = r + KG j.
template <int N0W, int KG, int ST, typename Emit>
__device__ __forceinline__ void column_levels(float2 z, float2 (&ring)[ColCfg<N0W, KG>::RING_TOTAL],
                                              const float2 (&lanefac)[ColCfg<N0W, KG>::M0 + 1],
                                              const float2* w0, Emit&& emit) {
  using CC = ColCfg<N0W, KG>;
  float2 cur[N0W];
  cur[0] = z;
  sfor<1, CC::M0 + 1>([&](auto U) {
    constexpr int u = U;
    constexpr int s = N0W >> u;
    constexpr int hp = CC::held(u - 1);
    constexpr int base = CC::ring_off(u) + (ST % s) * hp;
    if constexpr (u <= CC::G) {
      // one node per lane: i_u = r mod 2^u from i_{u-1} = r mod 2^{u-1}
      const float2 b = ring[base];
      const float2 d = cur[0];
      ring[base] = d;
      const float2 f = lanefac[u];
      cur[0] = make_float2(b.x + (f.x * d.x - f.y * d.y), b.y + (f.x * d.y + f.y * d.x));
    } else {
      float2 nxt[N0W];
      sfor<0, hp>([&](auto J) {
        constexpr int j = J;
        const float2 b = ring[base + j];
        float2 d = cur[j];
        ring[base + j] = d;
        if constexpr (KG > 1) {
          const float2 f = lanefac[u];
          d = make_float2(f.x * d.x - f.y * d.y, f.x * d.y + f.y * d.x);
        }
        const float2 t = twmul<KG * j * s, N0W>(d, w0);
        if constexpr (u == CC::M0) {
          emit(std::integral_constant<int, j>{}, cadd(b, t));
          emit(std::integral_constant<int, j + hp>{}, csub(b, t));
        } else {
          nxt[j] = cadd(b, t);
          nxt[j + hp] = csub(b, t);
        }
      });
      if constexpr (u < CC::M0) {
        sfor<0, 2 * hp>([&](auto K) { cur[K] = nxt[K]; });
      }
    }
  });
}

__device__ __forceinline__ void store_nt(float2* p, float2 v) {
  f2v t;
  t.x = v.x;
  t.y = v.y;
  __builtin_nontemporal_store(t, reinterpret_cast<f2v*>(p));
}

// Workgroup i runs on XCD i mod 8; give each XCD a contiguous block of tiles.
__device__ __forceinline__ int xcd_tile(int id, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, r = nb % kXcd;
  const int x = id % kXcd, j = id / kXcd;
  return x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

template <int N0W, int N1W, bool REAL, int KG>
struct TreeCfg {
  static constexpr int M0 = ilog2(N0W);
  static constexpr int QW = 64 / (N1W * KG);                // window columns per wave
  static constexpr int R = 64 / QW;                         // rows per row pass
  static constexpr int RING = N0W > 1 ? N0W / 2 : 1;        // ring period
  static constexpr int CR = R > RING ? R : RING;            // rows per chunk
  static constexpr int ZS = N1W + 1;                        // padded stride of one window column in LDS
  static constexpr int ZROW = QW * ZS;                      // float2 per chunk row in LDS
  static constexpr int LDS_FLOAT2 = CR * ZROW;
  static_assert(KG == 1 || KG < N0W, "a split stream needs KG < n0");
  static_assert(N1W * KG <= 64, "one wave must hold a whole window column");
};

// One tile of the forward tree: window columns [strip*QW, +QW) and window
// rows [slab*S, +S) of image b. w0, w1 point at the twiddle vectors (kernel
// arguments or a device table); zl is the wave's LDS buffer of
// TreeCfg::LDS_FLOAT2 elements.
template <int N0W, int N1W, bool REAL, int KG>
__device__ __forceinline__ void tree_fwd_tile(const void* __restrict__ xv, float2* __restrict__ y,
                                              const TreeGeom& g_in, const float2* __restrict__ w0,
                                              const float2* __restrict__ w1, int strip, int slab,
                                              int b, float2* __restrict__ zl) {
  using C = TreeCfg<N0W, N1W, REAL, KG>;
  using CC = ColCfg<N0W, KG>;
  const int lane = threadIdx.x;
  const TreeGeom g = uniform_copy(g_in);

  const int64_t q1_0 = (int64_t)strip * C::QW;
  const int64_t row0 = (int64_t)slab * g.S;
  const int64_t q0_end = min(row0 + (int64_t)g.S, g.P0);
  const int nrows = (int)(q0_end - row0) + N0W - 1;
  const int nchunks = (nrows + C::CR - 1) / C::CR;

  const float* xr = reinterpret_cast<const float*>(xv) + (REAL ? b * g.x_image_stride : 0);
  const float2* xc = reinterpret_cast<const float2*>(xv) + (REAL ? 0 : b * g.x_image_stride);
  float2* yimg = y + b * g.y_image_stride;

  // row-phase roles: lane (r, c) = input row r of the pass, window column c
  const int rp_r = lane / C::QW;
  const int rp_c = lane % C::QW;
  const int64_t rp_q1 = q1_0 + rp_c;
  // column-phase roles: lane (c, res, k1)
  const int cp_c = lane / (N1W * KG);
  const int cp_res = (lane / N1W) % KG;
  const int cp_k1 = lane % N1W;
  const int64_t cp_q1 = q1_0 + cp_c;
  const bool cp_ok = cp_q1 < g.P1;
  float2* ycol = yimg + cp_q1 * (N0W * N1W) + cp_res * N1W + cp_k1;
  const int64_t y_row_stride = g.P1 * (N0W * N1W);

  float2 lanefac[CC::M0 + 1];
  lanefac[0] = make_float2(1.f, 0.f);
  sfor<1, CC::M0 + 1>([&](auto U) {
    constexpr int u = U;
    if constexpr (KG > 1) {
      const int idx = (cp_res & ((1 << u) - 1)) * (N0W >> u);
      lanefac[u] = w0[idx];
    } else {
      lanefac[u] = make_float2(1.f, 0.f);
    }
  });

  float2 ring[CC::RING_TOTAL];
  sfor<0, CC::RING_TOTAL>([&](auto K) { ring[K] = make_float2(0.f, 0.f); });

  for (int c = 0; c < nchunks; ++c) {
    const int64_t crow = row0 + (int64_t)c * C::CR;

    // ---- row phase: CR rows x QW window columns of Z into LDS
    sfor<0, C::CR / C::R>([&](auto PS) {
      constexpr int ps = PS;
      const int64_t row = crow + ps * C::R + rp_r;
      const bool row_ok = row < g.N0;
      float2 v[N1W];
      sfor<0, N1W>([&](auto D) {
        constexpr int d = D;
        const int64_t col = rp_q1 + (N1W - 1 - d);
        const bool ok = row_ok && col < g.N1;
        if constexpr (REAL) {
          v[d] = make_float2(ok ? xr[row * g.N1 + col] : 0.f, 0.f);
        } else {
          v[d] = ok ? xc[row * g.N1 + col] : make_float2(0.f, 0.f);
        }
      });
      row_levels<N1W>(v, w1);
      if (g.scale != 1.0f) {
        sfor<0, N1W>([&](auto K) { v[K] = make_float2(v[K].x * g.scale, v[K].y * g.scale); });
      }
      float2* zrow = zl + (ps * C::R + rp_r) * C::ZROW + rp_c * C::ZS;
      sfor<0, N1W>([&](auto K) { zrow[K] = v[K]; });
    });
    __syncthreads();

    // ---- column phase: CR steps down the slab, one input row each
    sfor<0, C::CR>([&](auto STc) {
      constexpr int st = STc;
      const float2 z = zl[st * C::ZROW + cp_c * C::ZS + cp_k1];
      const int64_t q0 = crow + st - (N0W - 1);
      const bool store = (q0 >= row0) && (q0 < q0_end) && cp_ok;
      float2* dst = ycol + q0 * y_row_stride;
      if constexpr (N0W == 1) {
        if (store) store_nt(dst, z);
      } else {
        column_levels<N0W, KG, st % C::RING>(z, ring, lanefac, w0, [&](auto J, float2 v) {
          if (store) store_nt(dst + (KG * J) * N1W, v);
        });
      }
    });
    __syncthreads();
  }
}

template <int N0W, int N1W, bool REAL, int KG>
__global__ __launch_bounds__(64) void tree_fwd_kernel(const void* __restrict__ xv,
                                                      float2* __restrict__ y, TreeGeom g,
                                                      TwiddlesF32 tw) {
  using C = TreeCfg<N0W, N1W, REAL, KG>;
  __shared__ float2 zl[C::LDS_FLOAT2];
  int id = xcd_tile(blockIdx.x, gridDim.x);
  const int strip = id % g.nstrips;
  id /= g.nstrips;
  const int slab = id % g.nslabs;
  const int b = id / g.nslabs;
  tree_fwd_tile<N0W, N1W, REAL, KG>(xv, y, g, tw.w0, tw.w1, strip, slab, b, zl);
}

template <int N0W, int N1W, bool REAL>
hipError_t launch_one(const void* x, float2* y, const TreeGeom& g, const TwiddlesF32& tw,
                      hipStream_t stream) {
  const int64_t nb = (int64_t)g.batch * g.nslabs * g.nstrips;
  if constexpr (N0W >= 8 && N1W <= 32) {
    if (g.kg == 2) {
      hipLaunchKernelGGL((tree_fwd_kernel<N0W, N1W, REAL, 2>), dim3((unsigned)nb), dim3(64), 0,
                         stream, x, y, g, tw);
      return hipGetLastError();
    }
  }
  if (g.kg != 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((tree_fwd_kernel<N0W, N1W, REAL, 1>), dim3((unsigned)nb), dim3(64), 0, stream,
                     x, y, g, tw);
  return hipGetLastError();
}

// One translation unit per (n0, input type) instantiates launchers for every n1.
template <int N0W, bool REAL>
hipError_t launch_n0(int n1, const void* x, float2* y, const TreeGeom& g, const TwiddlesF32& tw,
                     hipStream_t s) {
  switch (n1) {
    case 1: return launch_one<N0W, 1, REAL>(x, y, g, tw, s);
    case 2: return launch_one<N0W, 2, REAL>(x, y, g, tw, s);
    case 4: return launch_one<N0W, 4, REAL>(x, y, g, tw, s);
    case 8: return launch_one<N0W, 8, REAL>(x, y, g, tw, s);
    case 16: return launch_one<N0W, 16, REAL>(x, y, g, tw, s);
    case 32: return launch_one<N0W, 32, REAL>(x, y, g, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tree

#define SWDFT_FWD_DECL(N0W, TAG) \
  hipError_t launch_tree_fwd_n0_##N0W##_##TAG(int, const void*, float2*, const TreeGeom&, \
                                             const TwiddlesF32&, hipStream_t);
SWDFT_FWD_DECL(1, r)
SWDFT_FWD_DECL(1, c)
SWDFT_FWD_DECL(2, r)
SWDFT_FWD_DECL(2, c)
SWDFT_FWD_DECL(4, r)
SWDFT_FWD_DECL(4, c)
SWDFT_FWD_DECL(8, r)
SWDFT_FWD_DECL(8, c)
SWDFT_FWD_DECL(16, r)
SWDFT_FWD_DECL(16, c)
SWDFT_FWD_DECL(32, r)
SWDFT_FWD_DECL(32, c)
#undef SWDFT_FWD_DECL

}  // namespace swdft
