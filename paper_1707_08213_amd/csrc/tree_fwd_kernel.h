// Fused forward 2D Tree SWDFT for gfx950.
//
// The tree of Sec. 4.2 is a row-column radix-2 decimation-in-time FFT whose
// nodes are indexed by window position. Row levels t = 1..m1 (Eq. (5)) build,
// for every position p1, the n1-point DFT Z[p0][q1][k1] of the row segment
// x[p0][q1 .. q1+n1-1]; column levels v = m1+1..m1+m0 (Eq. (6)) then build the
// n0-point DFT of each column of Z, which is the 2D DFT of the window. The
// final level is the output (Sec. 4.2, last paragraph).
//
// Mapping to the hardware (workgroups of WV wave64s, independent of each
// other):
//  * A workgroup owns a strip of QW = 64/(n1 KG) adjacent window columns and
//    a slab of S output rows of one image. Lane (c, k1) of the column phase
//    owns the stream Z[.][q1_0 + c][k1] and walks it down the slab one input
//    row per step. A stream may be split by k0 residue over KG lanes of a wave
//    and WV waves of the workgroup (KT = KG WV residues; see ColCfg and
//    TreeCfg), each part holding 1/KT of the nodes of every tree.
//  * Column phase (Eq. (6)), in registers: at row p a lane needs level u-1 of
//    its own tree (p) and of tree p - s_u, s_u = n0 / 2^u. It keeps the last
//    s_u positions of every level u-1 in a register ring (n0/(2 KT) complex
//    values per level and lane, m0 levels). Rows are processed in chunks whose length is a
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
//    consecutive windows (KG adjacent k0 rows for a split stream), i.e.
//    whole 128-byte lines from n1 KG >= 16 on, with non-temporal stores
//    (plain stores below that); the output is the only large HBM stream.
//  * The first n0-1 rows of a slab only prime the rings (their windows belong
//    to the previous slab); their outputs are not stored. Stores go through a
//    buffer resource per output row whose range ends at the strip's last
//    window (empty for priming rows): the hardware drops out-of-range lanes,
//    so the store stream has no exec-mask branches. Partial trees near
//    the top and left edges (Sec. 4.7) read zeros and are never stored.
//  * Occupancy and tile order: the host may cap the resident workgroups per
//    CU (extra dynamic LDS that the kernel does not touch). With one per CU
//    and a workgroup per whole column of its strip, the resident waves write
//    one band of consecutive output rows that moves down the image; when the
//    tiles need more than one round of resident workgroups they run in
//    dispatch order, so that each round covers one contiguous range of
//    strips. Otherwise workgroup ids are remapped so that each XCD (own L2)
//    gets a contiguous range of tiles: neighbouring strips share input
//    columns.
//  * Inputs of the next chunk are loaded (through a buffer resource that
//    returns zero past the image) before the column phase of the current
//    chunk, whose stores then separate the loads from their use: the wait
//    for the inputs never drains the output stores.
#pragma once
#include <type_traits>

#include "internal.h"
#include "swdft2d.h"

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

// Load a value that is the same for every lane of the wave, through the
// constant address space so that it is fetched by a scalar load into scalar
// registers. Used for twiddles, which live in the kernel arguments or in a
// device table that no kernel writes.
__device__ __forceinline__ float2 uload(const float2* p) {
  typedef const __attribute__((address_space(4))) float* const_ptr;
  const const_ptr q = (const_ptr)(reinterpret_cast<const float*>(p));
  return make_float2(q[0], q[1]);
}

// A 64-bit value known to be the same in every lane, kept in scalar registers.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t uniform_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
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

// a * b for complex a, b with every rounding written out: each part is one
// rounded product fed to one fused multiply-add, so that no choice is left
// to the compiler's contraction and every inlined copy of a butterfly (the
// unrolled steps of a chunk, the priming steps of a slab's first chunk, the
// other kernels that share these levels) rounds the same way.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
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
    return cmul(uload(w + IDX), d);
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
  // twiddle index of node r + KG j at level u (u > G), without the lane part
  static constexpr int tw_index(int u, int j) { return KG * j * (N0W >> u); }
  // uniform twiddles other than 1 and -i; at a split level these are folded
  // into a per-lane factor once per tile
  static constexpr bool folded(int u, int j) {
    return KG > 1 && u > G && tw_index(u, j) != 0 && 4 * tw_index(u, j) != N0W;
  }
  static constexpr int LW = N0W / 2 > 0 ? N0W / 2 : 1;  // held(u - 1) <= n0 / 2
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
// Where the uniform twiddle is not 1 or -i the product is precomputed per
// lane (lw[u][j]), so every node costs one complex multiply.
// emit(j, v) receives output k0 = r + KG j.
//
// T0 >= 0 marks row p as the T0-th row of a slab whose first window starts
// at that slab's first row. Level u of row p is then used by some window of
// the slab only if T0 >= n0 - s_u (it feeds the windows ending at rows p to
// p + s_u - 1), so the priming rows T0 < n0 - 1 compute only those levels,
// keep in the ring only the level values a later used node reads, and emit
// nothing. T0 = -1 computes every level.
template <int N0W, int KG, int ST, int T0 = -1, typename Emit>
__device__ __forceinline__ void column_levels(float2 z, float2 (&ring)[ColCfg<N0W, KG>::RING_TOTAL],
                                              const float2 (&lanefac)[ColCfg<N0W, KG>::M0 + 1],
                                              const float2 (&lw)[ColCfg<N0W, KG>::M0 + 1][ColCfg<N0W, KG>::LW],
                                              const float2* w0, Emit&& emit) {
  using CC = ColCfg<N0W, KG>;
  float2 cur[N0W];
  cur[0] = z;
  sfor<1, CC::M0 + 1>([&](auto U) {
    constexpr int u = U;
    constexpr int s = N0W >> u;
    constexpr int hp = CC::held(u - 1);
    constexpr int base = CC::ring_off(u) + (ST % s) * hp;
    constexpr bool level_in = T0 < 0 || T0 >= N0W - (N0W >> (u - 1));  // level u-1 used
    constexpr bool level_out = T0 < 0 || T0 >= N0W - s;                 // level u used
    if constexpr (!level_in) {
      // nothing of this level or above is used at this row
    } else if constexpr (!level_out) {
      // level u-1 is read again s_u rows later; level u is not needed yet
      sfor<0, hp>([&](auto J) { ring[base + J] = cur[J]; });
    } else if constexpr (u <= CC::G) {
      // one node per lane: i_u = r mod 2^u from i_{u-1} = r mod 2^{u-1}
      const float2 b = ring[base];
      const float2 d = cur[0];
      ring[base] = d;
      cur[0] = cadd(b, cmul(lanefac[u], d));
    } else {
      float2 nxt[N0W];
      sfor<0, hp>([&](auto J) {
        constexpr int j = J;
        const float2 b = ring[base + j];
        float2 d = cur[j];
        ring[base + j] = d;
        float2 t;
        if constexpr (CC::folded(u, j)) {
          t = cmul(lw[u][j], d);
        } else {
          if constexpr (KG > 1) d = cmul(lanefac[u], d);
          t = twmul<KG * j * s, N0W>(d, w0);
        }
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

// Buffer resource over [base, base + nbytes): a raw buffer store whose byte
// offset is at or past nbytes is dropped by the hardware. The tree stores its
// output through one such resource per output row and strip, so that lanes
// past the right edge and rows outside the slab need no branch.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t nbytes) {
  constexpr int kRawBufferFormat = 0x00020000;  // word 3 of a raw (untyped) gfx9 buffer
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)nbytes,
                                           kRawBufferFormat);
}

typedef unsigned u2v __attribute__((ext_vector_type(2)));

// A byte offset no buffer of this library reaches: a load there returns zero,
// a store there is dropped. Input resources span at most 128 rows (TreeCfg::CR)
// of at most SWDFT_MAX_ROW elements of 8 bytes, i.e. at most 2^31 bytes, and
// offsets past this value plus one chunk stay below 2^32.
constexpr uint32_t kOutOfRange = 0x80000000u;

// Input element at byte offset off of a buffer resource; zero past its end.
template <bool REAL>
__device__ __forceinline__ std::conditional_t<REAL, float, float2> load_buf(
    __amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (REAL) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
  } else {
    const u2v t = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
    return make_float2(__uint_as_float(t.x), __uint_as_float(t.y));
  }
}

// 8-byte store at byte offset off of a buffer resource, non-temporal by
// default.
template <bool NT = true>
__device__ __forceinline__ void store_buf(__amdgpu_buffer_rsrc_t r, uint32_t off, float2 v) {
  constexpr int kNonTemporal = 2;
  u2v t;
  t.x = __float_as_uint(v.x);
  t.y = __float_as_uint(v.y);
  __builtin_amdgcn_raw_buffer_store_b64(t, r, (int)off, 0, NT ? kNonTemporal : 0);
}

__device__ __forceinline__ void store_buf_nt(__amdgpu_buffer_rsrc_t r, uint32_t off, float2 v) {
  store_buf<true>(r, off, v);
}

// Rows of one chunk of steps that touch a row buffer: step st of a chunk that
// starts at input row crow is window row q = crow + st - lag, and only rows
// in [q_begin, q_end) are real (the others prime the rings or lie past the
// slab). [lo, lo + span) are those steps, as scalar values.
struct StepSpan {
  int lo;
  uint32_t span;
};

// Integer clamp (the min/max templates of the device headers may take a
// detour through double precision).
__device__ __forceinline__ int64_t clamp_i64(int64_t v, int64_t lo, int64_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

__device__ __forceinline__ StepSpan step_span(int64_t crow, int64_t q_begin, int64_t q_end, int lag,
                                              int steps) {
  const int lo = (int)uniform_u32((uint32_t)clamp_i64(q_begin + lag - crow, 0, steps));
  const int hi = (int)uniform_u32((uint32_t)clamp_i64(q_end + lag - crow, lo, steps));
  return StepSpan{lo, (uint32_t)(hi - lo)};
}

// Buffer resource of one row for step st: the row's address (an integer
// kept in scalar registers and advanced by one row per step by the caller,
// so a step spends a few scalar instructions on its resource; the tile's rate
// is bounded by a wave's instruction issue) and nbytes, or an empty range on
// the steps outside the span. The address of a step outside the span may lie
// outside the buffer; it is never dereferenced.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t step_rsrc(uint64_t addr, int st, StepSpan sp,
                                                            uint32_t nbytes) {
  return buf_rsrc((const void*)(uintptr_t)uniform_u64(addr),
                  uniform_u32((uint32_t)(st - sp.lo) < sp.span ? nbytes : 0u));
}

// Workgroup i runs on XCD i mod 8; give each XCD a contiguous block of tiles.
__device__ __forceinline__ int xcd_tile(int id, int nb) {
  constexpr int kXcd = 8;
  const int q = nb / kXcd, r = nb % kXcd;
  const int x = id % kXcd, j = id / kXcd;
  return x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

// Tile shape. KG lanes of a wave split a column stream by k0 residue; WV
// waves of a workgroup share one strip and split it further (residue
// r = lane residue + KG * wave), so KT = KG * WV. Each wave computes the
// row phase for CR / WV of the chunk's rows.
template <int N0W, int N1W, bool REAL, int KG, int WV = 1>
struct TreeCfg {
  static constexpr int M0 = ilog2(N0W);
  static constexpr int KT = KG * WV;                        // total split of a stream
  static constexpr int QW = 64 / (N1W * KG);                // window columns per strip
  static constexpr int R = 64 / QW;                         // rows per row pass of a wave
  static constexpr int RING = N0W > 1 ? N0W / 2 : 1;        // ring period
  static constexpr int CR = R * WV > RING ? R * WV : RING;  // rows per chunk
  static constexpr int PPW = CR / (R * WV);                 // row passes per wave and chunk
  static constexpr int ZS = N1W + 1;                        // padded stride of one window column in LDS
  static constexpr int ZROW = QW * ZS;                      // float2 per chunk row in LDS
  static constexpr int LDS_FLOAT2 = CR * ZROW;
  // One store instruction writes, per window, KG adjacent k0 rows of n1
  // complex64 values. Non-temporal stores are used when that covers whole
  // 128-byte lines (KG n1 >= 16); narrower rows (n1 <= 8 unsplit, n1 <= 4
  // split in two) take plain stores, so that L2 merges the k0 rows of a
  // line before it is written back (non-temporal partial lines reached
  // about 1 TB/s at 1024 x 1024 / 4 x 4).
  static constexpr bool NT_STORES = KG * N1W >= 16;
  static_assert(KT == 1 || KT < N0W, "a split stream needs KG * WV < n0");
  static_assert((int64_t)CR * SWDFT_MAX_ROW * 8 <= (int64_t)kOutOfRange,
                "one chunk of input rows must stay addressable with 32-bit offsets");
  static_assert(N1W * KG <= 64, "one wave must hold a whole window column");
};

// One tile of the forward tree: window columns [strip*QW, +QW) and window
// rows [slab*S, +S) of image b. w0, w1 point at the twiddle vectors (kernel
// arguments or a device table); zl is the wave's LDS buffer of
// TreeCfg::LDS_FLOAT2 elements.
template <int N0W, int N1W, bool REAL, int KG, int WV = 1>
__device__ __forceinline__ void tree_fwd_tile(const void* __restrict__ xv, float2* __restrict__ y,
                                              const TreeGeom& g_in, const float2* __restrict__ w0,
                                              const float2* __restrict__ w1, int strip, int slab,
                                              int b, float2* __restrict__ zl) {
  using C = TreeCfg<N0W, N1W, REAL, KG, WV>;
  using CC = ColCfg<N0W, C::KT>;
  const int lane = threadIdx.x % 64;
  const int wv = WV > 1 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64) : 0;
  const TreeGeom g = uniform_copy(g_in);

  const int64_t q1_0 = (int64_t)strip * C::QW;
  const int64_t row0 = (int64_t)slab * g.S;
  const int64_t q0_end = min(row0 + (int64_t)g.S, g.P0);
  const int nrows = (int)(q0_end - row0) + N0W - 1;
  const int nchunks = (nrows + C::CR - 1) / C::CR;

  using XT = std::conditional_t<REAL, float, float2>;
  constexpr int EB = (int)sizeof(XT);
  const XT* ximg = reinterpret_cast<const XT*>(xv) + b * g.x_image_stride;
  float2* yimg = y + b * g.y_image_stride;

  // row-phase roles: lane (r, c) = input row r of the pass, window column c
  const int rp_r = lane / C::QW;
  const int rp_c = lane % C::QW;
  const int64_t rp_q1 = q1_0 + rp_c;
  // byte offset of the lane's input x[r][q1 + n1 - 1 - d] within a chunk of
  // rows; columns past the image edge read zero (Sec. 4.7). Kept in registers
  // up to n1 = 32; the 64 of n1 = 64 are recomputed at each load.
  constexpr bool kKeepOffsets = N1W <= 32;
  uint32_t x_off_keep[kKeepOffsets ? N1W : 1];
  auto x_off_of = [&](int d) __attribute__((always_inline)) -> uint32_t {
    const int64_t col = rp_q1 + (N1W - 1 - d);
    return col < g.N1 ? (uint32_t)(((int64_t)rp_r * g.N1 + col) * EB) : kOutOfRange;
  };
  if constexpr (kKeepOffsets) sfor<0, N1W>([&](auto D) { x_off_keep[D] = x_off_of(D); });
  auto x_off = [&](auto D) __attribute__((always_inline)) -> uint32_t {
    if constexpr (kKeepOffsets) {
      return x_off_keep[D];
    } else {
      return x_off_of(D);
    }
  };
  // Raw inputs of this wave's passes of one chunk (rows crow + (wv * PPW +
  // ps) * R + r), loaded a chunk ahead so that their latency hides behind the
  // column phase of the previous chunk (up to n1 = 32; at n1 = 64 the
  // registers are worth more to the rings, and the loads come right before
  // the row phase). Rows past the image bottom lie outside the resource and
  // read zero.
  constexpr bool kPrefetch = N1W <= 32;
  constexpr int PASSES = C::PPW;
  XT xin[PASSES][N1W];
  auto load_chunk = [&](int64_t crow) __attribute__((always_inline)) {
    // scalar values, so that the loads need no loop over distinct
    // resources (the device min template goes through double precision)
    const int64_t rows = clamp_i64(g.N0 - crow, 0, C::CR);
    const auto rs = buf_rsrc(
        (const void*)(uintptr_t)uniform_u64((uint64_t)(uintptr_t)(ximg + (rows > 0 ? crow : 0) * g.N1)),
        uniform_u32((uint32_t)(rows * g.N1 * EB)));
    const uint32_t wave_off = (uint32_t)(wv * C::PPW * C::R * g.N1 * EB);
    sfor<0, PASSES>([&](auto PS) {
      constexpr int ps = PS;
      sfor<0, N1W>([&](auto D) {
        constexpr int d = D;
        xin[ps][d] = load_buf<REAL>(rs, x_off(D) + wave_off + (uint32_t)(ps * C::R * g.N1 * EB));
      });
    });
  };

  // column-phase roles: lane (c, res, k1); the stream residue is shared
  // between the lane (KG) and the wave (WV)
  const int cp_c = lane / (N1W * KG);
  const int cp_res = (lane / N1W) % KG + KG * wv;
  const int cp_k1 = lane % N1W;
  // Output of one row of the strip: QW windows of n0*n1 values from ystrip +
  // q0 * row_bytes; only the first strip_bytes exist (the last strip of a
  // row may be partial).
  float2* ystrip = yimg + q1_0 * (N0W * N1W);
  const uint64_t row_bytes = (uint64_t)g.P1 * (N0W * N1W * sizeof(float2));
  const uint32_t strip_bytes = uniform_u32(
      (uint32_t)(min((int64_t)C::QW, g.P1 - q1_0) * (N0W * N1W * (int)sizeof(float2))));
  const uint32_t lane_off =
      (uint32_t)((cp_c * (N0W * N1W) + cp_res * N1W + cp_k1) * (int)sizeof(float2));

  float2 lanefac[CC::M0 + 1];
  lanefac[0] = make_float2(1.f, 0.f);
  sfor<1, CC::M0 + 1>([&](auto U) {
    constexpr int u = U;
    if constexpr (C::KT > 1) {
      const int idx = (cp_res & ((1 << u) - 1)) * (N0W >> u);
      lanefac[u] = w0[idx];
    } else {
      lanefac[u] = make_float2(1.f, 0.f);
    }
  });

  float2 lw[CC::M0 + 1][CC::LW];
  sfor<1, CC::M0 + 1>([&](auto U) {
    constexpr int u = U;
    sfor<0, CC::LW>([&](auto J) {
      constexpr int j = J;
      if constexpr (CC::folded(u, j)) lw[u][j] = cmul(lanefac[u], uload(w0 + CC::tw_index(u, j)));
    });
  });

  float2 ring[CC::RING_TOTAL];
  sfor<0, CC::RING_TOTAL>([&](auto K) { ring[K] = make_float2(0.f, 0.f); });

  // ---- row phase: the CR rows x QW window columns of Z of one chunk, from
  // the raw inputs in xin, into LDS
  auto row_phase = [&]() __attribute__((always_inline)) {
    sfor<0, PASSES>([&](auto PS) {
      constexpr int ps = PS;
      float2 v[N1W];
      sfor<0, N1W>([&](auto D) {
        constexpr int d = D;
        if constexpr (REAL) {
          v[d] = make_float2(xin[ps][d], 0.f);
        } else {
          v[d] = xin[ps][d];
        }
      });
      row_levels<N1W>(v, w1);
      if (g.scale != 1.0f) {
        sfor<0, N1W>([&](auto K) { v[K] = make_float2(v[K].x * g.scale, v[K].y * g.scale); });
      }
      float2* zrow = zl + ((wv * C::PPW + ps) * C::R + rp_r) * C::ZROW + rp_c * C::ZS;
      sfor<0, N1W>([&](auto K) { zrow[K] = v[K]; });
    });
  };

  // The loop is rotated: iteration c issues the loads of chunk c+1, runs the
  // column phase of chunk c (whose stores then sit between those loads and
  // their use) and only then the row phase of chunk c+1, so the wait for the
  // inputs never has to drain the output stores.
  load_chunk(row0);
  row_phase();
  __syncthreads();
  // One chunk: c, and FIRST for the slab's first chunk, whose step st is the
  // slab's row st and whose priming steps (st < n0 - 1) compute only the
  // column levels that a window of the slab uses (column_levels). The first
  // chunk is peeled off the loop, so the loop holds one copy of the steps.
  auto chunk = [&](int c, auto FIRST) __attribute__((always_inline)) {
    const int64_t crow = row0 + (int64_t)c * C::CR;
    // (the loads of a chunk past the image bottom read zeros and touch no
    // memory; none is issued after the slab's last chunk, whose wave would
    // otherwise wait for them before it ends)
    if constexpr (kPrefetch) {
      if (c + 1 < nchunks) load_chunk(crow + C::CR);
    }
    __builtin_amdgcn_sched_barrier(0);

    // ---- column phase: CR steps down the slab, one input row each. The Z
    // value of a step is read from LDS kLdsAhead steps before it is used.
    constexpr int kLdsAhead = 2;
    const float2* zcol = zl + cp_c * C::ZS + cp_k1;
    float2 zq[C::CR];
    sfor<0, (kLdsAhead < C::CR ? kLdsAhead : C::CR)>([&](auto K) { zq[K] = zcol[K * C::ZROW]; });
    // Step st writes window row q0 = crow + st - (n0 - 1) when row0 <= q0 <
    // q0_end; the other steps prime the rings (or run past the slab) and get
    // an empty resource. row_addr is the address of row q0 of step 0 (as an
    // integer: the priming rows of the top slab lie before y).
    const StepSpan sp = step_span(crow, row0, q0_end, N0W - 1, C::CR);
    uint64_t row_addr = uniform_u64((uint64_t)(uintptr_t)ystrip +
                                    (uint64_t)(crow - (N0W - 1)) * row_bytes);
    // Steps past the slab's last row (in its last chunk; the short slabs of
    // small images end early in their only chunk) would only prime rings that
    // are never used. Long chunks (CR >= 32 rows, the split and multi-wave
    // tiles) skip them in blocks of SB steps with a uniform branch; short
    // chunks run whole (a branch per few light steps measurably slowed them:
    // 1024^2 / 8 x 8, 90 -> 97 us).
    constexpr bool kSkip = C::CR >= 32;
    constexpr int SB = kSkip ? 8 : C::CR;
    const int live = kSkip ? min(C::CR, nrows - c * C::CR) : C::CR;
    sfor<0, C::CR / SB>([&](auto BLK) {
      if (!kSkip || BLK * SB < live) {
        sfor<0, SB>([&](auto SS) {
          constexpr int st = BLK * SB + SS;
          if constexpr (st + kLdsAhead < C::CR)
            zq[st + kLdsAhead] = zcol[(st + kLdsAhead) * C::ZROW];
          __builtin_amdgcn_sched_barrier(0);  // keep the read ahead of this step's work
          const float2 z = zq[st];
          // A priming step of the first chunk may only keep z in a ring for
          // the next chunk; the compiler may then sink its LDS read past the
          // barrier below, where another wave's row phase already overwrites
          // the row. Taking z here as an operand keeps the read in its step.
          if constexpr (FIRST && WV > 1) asm volatile("" ::"v"(z.x), "v"(z.y));
          const auto out = step_rsrc(row_addr, st, sp, strip_bytes);
          row_addr += row_bytes;
          if constexpr (N0W == 1) {
            store_buf<C::NT_STORES>(out, lane_off, z);
          } else {
            column_levels<N0W, C::KT, st % C::RING, (FIRST ? st : -1)>(
                z, ring, lanefac, lw, w0, [&](auto J, float2 v) {
                  store_buf<C::NT_STORES>(
                      out, lane_off + (C::KT * J) * N1W * (int)sizeof(float2), v);
                });
          }
        });
      }
    });
    __syncthreads();
    if (c + 1 < nchunks) {
      if constexpr (!kPrefetch) load_chunk(crow + C::CR);
      row_phase();
      __syncthreads();
    }
  };
  chunk(0, std::true_type{});
  for (int c = 1; c < nchunks; ++c) chunk(c, std::false_type{});
}

template <int N0W, int N1W, bool REAL, int KG, int WV>
__global__ __launch_bounds__(64 * WV) void tree_fwd_kernel(const void* __restrict__ xv,
                                                           float2* __restrict__ y, TreeGeom g,
                                                           TwiddlesF32 tw) {
  using C = TreeCfg<N0W, N1W, REAL, KG, WV>;
  __shared__ float2 zl[C::LDS_FLOAT2];
  int id = g.order ? (int)blockIdx.x : xcd_tile(blockIdx.x, gridDim.x);
  const int strip = id % g.nstrips;
  id /= g.nstrips;
  const int slab = id % g.nslabs;
  const int b = id / g.nslabs;
  tree_fwd_tile<N0W, N1W, REAL, KG, WV>(xv, y, g, tw.w0, tw.w1, strip, slab, b, zl);
}

// Dynamic LDS that caps the resident workgroups per CU at wpc: the
// workgroup's total LDS is set midway between lds_cu/(wpc+1) and
// lds_cu/wpc. The kernel does not touch it.
inline unsigned occupancy_lds(int wpc, int lds_cu, unsigned static_lds) {
  if (wpc <= 0 || lds_cu <= 0) return 0u;
  const unsigned want = (unsigned)(lds_cu / wpc + lds_cu / (wpc + 1)) / 2u;
  return want > static_lds ? want - static_lds : 0u;
}

// Two waves per strip exist for n0 >= 16 (where one wave per CU is the
// default and the wave's issue rate bounds the tile), and for n0 = 8 with
// two-lane streams (small images: four residues per stream).
constexpr bool tree_has_wv2(int n0, int kg) {
  return (n0 >= 16 && kg * 2 < n0) || (n0 == 8 && kg == 2);
}

// Lanes per stream of the n0 = 64 kernels: as many as one wave's 64 lanes
// allow (n1 * KG <= 64), at most 8. The register rings then hold 68 (KG = 8),
// 80 (KG = 4) or 112 (KG = 2) complex values per lane instead of the 192 of an
// unsplit stream. n0 = 64 is built for this split only.
constexpr int tree_kg64(int n1) { return n1 >= 64 ? 1 : (64 / n1 > 8 ? 8 : 64 / n1); }

// Lane splits built for each window shape.
constexpr bool tree_kg_built(int n0, int n1, int kg) {
  return n0 == 64 ? kg == tree_kg64(n1) : (kg == 1 || (kg == 2 && n0 >= 8 && n1 <= 32));
}

// Waves per strip built for each split: one wave unless the stream would
// stay whole (n0 = 64, n1 = 64, whose rings then need two waves), two where
// tree_has_wv2 allows.
constexpr bool tree_wv_built(int n0, int kg, int wv) {
  return wv == 1 ? (n0 < 64 || kg > 1)
                 : wv == 2 && tree_has_wv2(n0, kg);
}

template <int N0W, int N1W, bool REAL, int KG, int WV>
hipError_t launch_cfg(const void* x, float2* y, const TreeGeom& g, const TwiddlesF32& tw,
                      hipStream_t stream) {
  const int64_t nb = (int64_t)g.batch * g.nslabs * g.nstrips;
  const unsigned pad = occupancy_lds(
      g.wpc, g.lds_cu, TreeCfg<N0W, N1W, REAL, KG, WV>::LDS_FLOAT2 * (unsigned)sizeof(float2));
  hipLaunchKernelGGL((tree_fwd_kernel<N0W, N1W, REAL, KG, WV>), dim3((unsigned)nb), dim3(64 * WV),
                     pad, stream, x, y, g, tw);
  return hipGetLastError();
}

template <int N0W, int N1W, bool REAL, int KG>
hipError_t launch_kg(const void* x, float2* y, const TreeGeom& g, const TwiddlesF32& tw,
                     hipStream_t stream) {
  if constexpr (tree_wv_built(N0W, KG, 2)) {
    if (g.wv == 2) return launch_cfg<N0W, N1W, REAL, KG, 2>(x, y, g, tw, stream);
  }
  if constexpr (tree_wv_built(N0W, KG, 1)) {
    if (g.wv == 1) return launch_cfg<N0W, N1W, REAL, KG, 1>(x, y, g, tw, stream);
  }
  return hipErrorInvalidValue;
}

template <int N0W, int N1W, bool REAL>
hipError_t launch_one(const void* x, float2* y, const TreeGeom& g, const TwiddlesF32& tw,
                      hipStream_t stream) {
  if constexpr (tree_kg_built(N0W, N1W, 1)) {
    if (g.kg == 1) return launch_kg<N0W, N1W, REAL, 1>(x, y, g, tw, stream);
  }
  if constexpr (tree_kg_built(N0W, N1W, 2)) {
    if (g.kg == 2) return launch_kg<N0W, N1W, REAL, 2>(x, y, g, tw, stream);
  }
  if constexpr (tree_kg_built(N0W, N1W, 4)) {
    if (g.kg == 4) return launch_kg<N0W, N1W, REAL, 4>(x, y, g, tw, stream);
  }
  if constexpr (tree_kg_built(N0W, N1W, 8)) {
    if (g.kg == 8) return launch_kg<N0W, N1W, REAL, 8>(x, y, g, tw, stream);
  }
  return hipErrorInvalidValue;
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
    case 64: return launch_one<N0W, 64, REAL>(x, y, g, tw, s);
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
SWDFT_FWD_DECL(64, r)
SWDFT_FWD_DECL(64, c)
#undef SWDFT_FWD_DECL

}  // namespace swdft
