// Dense per-window 2D SWDFT on the gfx950 matrix cores:
//   Y_w = F_n0 X_w F_n1^T   for every n0 x n1 window X_w,
// F_n[k][j] = Omega[(j k) mod n] (the twiddle vectors of Sec. 4.2). This is
// the direct product form of Eq. (3)-(4) (a row DFT then a column DFT per
// window) evaluated as dense matrix products, the alternative the tree is
// compared with; nothing is shared between windows except that the row
// product of an input row (X_w F_n1^T restricted to that row) is formed once
// and read by the n0 windows that contain the row.
//
// Precision: every FP32 operand a is split into bf16 parts a = a_hi + a_lo
// (a_hi = bf16(a), a_lo = bf16(a - a_hi), both round-to-nearest-even) and a
// product a*b is formed as a_hi b_hi + a_hi b_lo + a_lo b_hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation (the a_lo b_lo term and the
// residue of the split are dropped: about 2^-16 relative per product).
//
// Complex products are real products of block matrices,
//   [Re C]   [Re A  -Im A] [Re B]
//   [Im C] = [Im A   Re A] [Im B],
// with the K index ordered (re/im, j) and, for the column product, the M index
// interleaved (k0, re/im) so that each lane's four accumulator rows hold the
// real and imaginary parts of two k0 values for one output column.
//
// Wave layout: one wave64 owns NC = max(16, n1) output columns c = (q1, k1)
// (16/n1 windows, or one window split in two 16-column blocks when n1 = 32)
// and a slab of S window rows. Per 16 input rows it forms Z = X F_n1^T on the
// matrix cores (M = 16 rows, K = (re/im, j1), N = (re/im, k1)), splits Z into
// bf16 hi/lo and stores it in an LDS ring indexed by row (row fastest, so one
// lane's eight consecutive rows are one run). Per window row q0 it forms
// Y = F_n0 Z[q0 .. q0+n0-1] (M = (k0, re/im), K = (re/im, j0), N = 16
// columns) and stores complex64 results. The run start q0 + 8 g moves by one
// row per step; steps are unrolled by 8 so each run's alignment is a
// compile-time constant and it is read with the widest aligned LDS loads
// (one b128, two b64, four b32, or five b32 and funnel shifts).
#pragma once
#include <type_traits>

#include "internal.h"

namespace swdft {
namespace dense {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

__device__ __forceinline__ void split(float v, __bf16& hi, __bf16& lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

__device__ __forceinline__ f32x4 mma(const bf16x8& a, const bf16x8& b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// acc += A * B with both operands split hi/lo (three products).
__device__ __forceinline__ f32x4 mma3(const bf16x8& ahi, const bf16x8& alo, const bf16x8& bhi,
                                      const bf16x8& blo, f32x4 c) {
  c = mma(ahi, bhi, c);
  c = mma(ahi, blo, c);
  c = mma(alo, bhi, c);
  return c;
}

__device__ __forceinline__ bf16x8 u4_to_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// Eight consecutive bf16 starting at p, whose element offset is = AL (mod 8)
// relative to a 16-byte boundary. Reads never go below p - 1 or above p + 8.
template <int AL>
__device__ __forceinline__ bf16x8 load_run(const __bf16* p) {
  u32x4 r;
  if constexpr (AL == 0) {
    r = *reinterpret_cast<const u32x4*>(p);
  } else if constexpr (AL == 4) {
    const uint2 a = *reinterpret_cast<const uint2*>(p);
    const uint2 b = *reinterpret_cast<const uint2*>(p + 4);
    r = u32x4{a.x, a.y, b.x, b.y};
  } else if constexpr ((AL & 1) == 0) {
    const unsigned* q = reinterpret_cast<const unsigned*>(p);
    r = u32x4{q[0], q[1], q[2], q[3]};
  } else {
    const unsigned* q = reinterpret_cast<const unsigned*>(p - 1);
    const unsigned w0 = q[0], w1 = q[1], w2 = q[2], w3 = q[3], w4 = q[4];
    r = u32x4{__builtin_amdgcn_alignbit(w1, w0, 16), __builtin_amdgcn_alignbit(w2, w1, 16),
              __builtin_amdgcn_alignbit(w3, w2, 16), __builtin_amdgcn_alignbit(w4, w3, 16)};
  }
  return u4_to_bf(r);
}

// One output value. Non-temporal where a store instruction covers whole
// 128-byte lines (16 consecutive k1 per window, n1 >= 16); for n1 = 8 a line
// is two k0 rows written by two instructions, and plain stores let L2 merge
// them before the write-back.
template <bool NT>
__device__ __forceinline__ void store_out(float2* p, float re, float im) {
  f2v t;
  t.x = re;
  t.y = im;
  if constexpr (NT) {
    __builtin_nontemporal_store(t, reinterpret_cast<f2v*>(p));
  } else {
    *reinterpret_cast<f2v*>(p) = t;
  }
}

template <int N0W, int N1W, bool REAL>
struct DenseCfg {
  static constexpr int NC = N1W > 16 ? N1W : 16;          // output columns per wave
  static constexpr int NB = NC / 16;                       // 16-column blocks
  static constexpr int QW = NC / N1W;                      // window columns per wave
  static constexpr int MT2 = 2 * N0W / 16;                 // M tiles, column product
  static constexpr int K2 = 2 * N0W;                       // K of the column product
  static constexpr int KB2 = (K2 + 31) / 32;               // K blocks (zero padded)
  static constexpr int K1 = REAL ? N1W : 2 * N1W;          // K of the row product
  static constexpr int KB1 = (K1 + 31) / 32;
  static constexpr int NT1 = 2 * N1W / 16;                 // N tiles of the row product
  static constexpr int RL = N0W > 16 ? 64 : 32;            // LDS ring rows
  static constexpr int RLP = RL + 16;                      // + 8 guard each side
  static constexpr int LOOK = (N0W - 1 + 15) / 16;         // row chunks ahead of windows
  static constexpr int LDS_BF16 = 2 * 2 * NC * RLP;
  static_assert(N0W >= 8 && N1W >= 8, "dense path needs n0, n1 >= 8");
  static_assert(16 * (LOOK + 1) <= RL, "ring too short");
};

template <int N0W, int N1W, bool REAL>
__device__ __forceinline__ __bf16* zslot(__bf16* zr, int ri, int hl, int c, int e) {
  using C = DenseCfg<N0W, N1W, REAL>;
  return zr + (((ri * 2 + hl) * C::NC + c) * C::RLP + e);
}

// One tile of the dense variant: window columns [strip*QW, +QW) and window
// rows [slab*S, +S) of image b. zr is the wave's LDS ring of
// DenseCfg::LDS_BF16 elements (16-byte aligned).
template <int N0W, int N1W, bool REAL>
__device__ __forceinline__ void dense_fwd_tile(const void* __restrict__ xv, float2* __restrict__ y,
                                               const DenseGeom& g_in, const float2* __restrict__ w0,
                                               const float2* __restrict__ w1, int strip, int slab,
                                               int b, __bf16* __restrict__ zr) {
  using C = DenseCfg<N0W, N1W, REAL>;
  const int lane = threadIdx.x;
  const int l16 = lane & 15;
  const int lg = lane >> 4;
  DenseGeom g;
  {
    struct Words { int w[sizeof(DenseGeom) / 4]; };
    const Words in = __builtin_bit_cast(Words, g_in);
    Words out;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(DenseGeom) / 4); ++i)
      out.w[i] = __builtin_amdgcn_readfirstlane(in.w[i]);
    g = __builtin_bit_cast(DenseGeom, out);
  }
  const int64_t q1_0 = (int64_t)strip * C::QW;
  const int64_t Q = (int64_t)slab * g.S;                  // first window row (multiple of 16)
  const int64_t q0_end = min(Q + (int64_t)g.S, g.P0);

  const float* xr = reinterpret_cast<const float*>(xv) + (REAL ? b * g.x_image_stride : 0);
  const float2* xc = reinterpret_cast<const float2*>(xv) + (REAL ? 0 : b * g.x_image_stride);
  float2* yimg = y + b * g.y_image_stride;

  // ---- constant operands: column product A (F_n0 blocks), row product B (F_n1 blocks)
  bf16x8 a2hi[C::MT2][C::KB2], a2lo[C::MT2][C::KB2];
  sfor<0, C::MT2>([&](auto MT) {
    sfor<0, C::KB2>([&](auto KB) {
      const int m = 16 * MT + l16;
      const int k0 = m >> 1, ro = m & 1;
      sfor<0, 8>([&](auto I) {
        const int kidx = 32 * KB + 8 * lg + I;
        float v = 0.f;
        if (kidx < C::K2) {
          const int ri = kidx / N0W, j0 = kidx % N0W;
          const float2 w = w0[(j0 * k0) & (N0W - 1)];
          v = ro == 0 ? (ri == 0 ? w.x : -w.y) : (ri == 0 ? w.y : w.x);
        }
        __bf16 h, l;
        split(v, h, l);
        a2hi[MT][KB][(int)I] = h;
        a2lo[MT][KB][(int)I] = l;
      });
    });
  });
  bf16x8 b1hi[C::NT1][C::KB1], b1lo[C::NT1][C::KB1];
  sfor<0, C::NT1>([&](auto NT) {
    sfor<0, C::KB1>([&](auto KB) {
      const int n = 16 * NT + l16;
      const int ro = n / N1W, k1 = n % N1W;
      sfor<0, 8>([&](auto I) {
        const int kidx = 32 * KB + 8 * lg + I;
        float v = 0.f;
        if (kidx < C::K1) {
          const int ri = kidx / N1W, j1 = kidx % N1W;
          const float2 w = w1[(j1 * k1) & (N1W - 1)];
          v = ri == 0 ? (ro == 0 ? w.x : w.y) : (ro == 0 ? -w.y : w.x);
        }
        __bf16 h, l;
        split(v, h, l);
        b1hi[NT][KB][(int)I] = h;
        b1lo[NT][KB][(int)I] = l;
      });
    });
  });

  // ---- row product for 16 input rows starting at row r0: Z into the ring
  auto row_chunk = [&](int64_t r0) {
    const int64_t row = r0 + l16;  // A operand: lane row l16, K group lg
    const bool row_ok = row < g.N0;
    sfor<0, C::QW>([&](auto WQ) {
      const int64_t q1 = q1_0 + WQ;
      bf16x8 ahi[C::KB1], alo[C::KB1];
      sfor<0, C::KB1>([&](auto KB) {
        const int kbase = 32 * KB + 8 * lg;  // multiple of 8: one re or im run
        const int ri = kbase / N1W, j1b = kbase % N1W;
        const bool live = kbase < C::K1;
        sfor<0, 8>([&](auto I) {
          const int64_t col = q1 + j1b + I;
          const bool ok = live && row_ok && col < g.N1;
          float v = 0.f;
          if constexpr (REAL) {
            v = ok ? xr[row * g.N1 + col] : 0.f;
          } else {
            const float2 t = ok ? xc[row * g.N1 + col] : make_float2(0.f, 0.f);
            v = ri == 0 ? t.x : t.y;
          }
          __bf16 h, l;
          split(v, h, l);
          ahi[KB][(int)I] = h;
          alo[KB][(int)I] = l;
        });
      });
      sfor<0, C::NT1>([&](auto NT) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        sfor<0, C::KB1>([&](auto KB) {
          acc = mma3(ahi[KB], alo[KB], b1hi[NT][KB], b1lo[NT][KB], acc);
        });
        // lane holds Z_ri[rows r0 + 4 lg + i][column n = 16 NT + l16]
        const int n = 16 * NT + l16;
        const int ro = n / N1W, k1 = n % N1W;
        const int c = WQ * N1W + k1;
        const int slot = (int)((r0 + 4 * lg) & (C::RL - 1));
        __bf16 hi[4], lo[4];
        sfor<0, 4>([&](auto I) { split(acc[(int)I] * g.scale, hi[(int)I], lo[(int)I]); });
        uint2 ph, pl;
        __builtin_memcpy(&ph, hi, 8);
        __builtin_memcpy(&pl, lo, 8);
        *reinterpret_cast<uint2*>(zslot<N0W, N1W, REAL>(zr, ro, 0, c, 8 + slot)) = ph;
        *reinterpret_cast<uint2*>(zslot<N0W, N1W, REAL>(zr, ro, 1, c, 8 + slot)) = pl;
        if (slot < 8) {
          *reinterpret_cast<uint2*>(zslot<N0W, N1W, REAL>(zr, ro, 0, c, 8 + C::RL + slot)) = ph;
          *reinterpret_cast<uint2*>(zslot<N0W, N1W, REAL>(zr, ro, 1, c, 8 + C::RL + slot)) = pl;
        }
      });
    });
  };

  const int nchunks = (int)((q0_end - Q + 15) / 16);
  sfor<0, C::LOOK>([&](auto L) { row_chunk(Q + 16 * L); });

  for (int wc = 0; wc < nchunks; ++wc) {
    const int64_t wq = Q + 16 * (int64_t)wc;
    row_chunk(wq + 16 * C::LOOK);
    __syncthreads();
    sfor<0, 16>([&](auto ST) {
      constexpr int st = ST;
      const int64_t q0 = wq + st;
      const bool row_live = q0 < q0_end;
      sfor<0, C::NB>([&](auto NBc) {
        const int c = 16 * NBc + l16;
        // B operand runs: K index 32 kb + 8 lg + i = (re/im, j0); rows q0 + j0
        bf16x8 bhi[C::KB2], blo[C::KB2];
        sfor<0, C::KB2>([&](auto KB) {
          const int kbase = 32 * KB + 8 * lg;
          if (kbase < C::K2) {
            const int ri = kbase / N0W, j0b = kbase % N0W;
            const int slot = (int)((wq + j0b) & (C::RL - 1)) + st;  // run start, mod RL below
            const int s = slot & (C::RL - 1);
            bhi[KB] = load_run<(st & 7)>(zslot<N0W, N1W, REAL>(zr, ri, 0, c, 8 + s));
            blo[KB] = load_run<(st & 7)>(zslot<N0W, N1W, REAL>(zr, ri, 1, c, 8 + s));
          } else {
            bhi[KB] = bf16x8{};
            blo[KB] = bf16x8{};
          }
        });
        const int64_t q1 = q1_0 + (c / N1W);
        const int k1 = c % N1W;
        const bool ok = row_live && q1 < g.P1;
        float2* dst = yimg + ((q0 * g.P1 + q1) * N0W) * N1W + k1;
        sfor<0, C::MT2>([&](auto MT) {
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
          sfor<0, C::KB2>([&](auto KB) {
            acc = mma3(a2hi[MT][KB], a2lo[MT][KB], bhi[KB], blo[KB], acc);
          });
          // rows 16 MT + 4 lg + i = (k0, re/im) interleaved: two k0 per lane
          if (ok) {
            const int k0a = 8 * MT + 2 * lg;
            store_out<(N1W >= 16)>(dst + k0a * N1W, acc[0], acc[1]);
            store_out<(N1W >= 16)>(dst + (k0a + 1) * N1W, acc[2], acc[3]);
          }
        });
      });
    });
    __syncthreads();
  }
}

template <int N0W, int N1W, bool REAL>
__global__ __launch_bounds__(64) void dense_fwd_kernel(const void* __restrict__ xv,
                                                       float2* __restrict__ y, DenseGeom g,
                                                       TwiddlesF32 tw) {
  using C = DenseCfg<N0W, N1W, REAL>;
  __shared__ __attribute__((aligned(16))) __bf16 zr[C::LDS_BF16];
  int id = blockIdx.x;
  const int strip = id % g.nstrips;
  id /= g.nstrips;
  const int slab = id % g.nslabs;
  const int b = id / g.nslabs;
  dense_fwd_tile<N0W, N1W, REAL>(xv, y, g, tw.w0, tw.w1, strip, slab, b, zr);
}

template <int N0W, int N1W, bool REAL>
hipError_t launch_one(const void* x, float2* y, const DenseGeom& g, const TwiddlesF32& tw,
                      hipStream_t stream) {
  const int64_t nb = (int64_t)g.batch * g.nslabs * g.nstrips;
  hipLaunchKernelGGL((dense_fwd_kernel<N0W, N1W, REAL>), dim3((unsigned)nb), dim3(64), 0, stream,
                     x, y, g, tw);
  return hipGetLastError();
}

template <bool REAL>
hipError_t launch(int n0, int n1, const void* x, float2* y, const DenseGeom& g,
                  const TwiddlesF32& tw, hipStream_t s) {
#define SWDFT_DCASE(A, B) \
  if (n0 == A && n1 == B) return launch_one<A, B, REAL>(x, y, g, tw, s);
  SWDFT_DCASE(8, 8)
  SWDFT_DCASE(8, 16)
  SWDFT_DCASE(8, 32)
  SWDFT_DCASE(16, 8)
  SWDFT_DCASE(16, 16)
  SWDFT_DCASE(16, 32)
  SWDFT_DCASE(32, 8)
  SWDFT_DCASE(32, 16)
  SWDFT_DCASE(32, 32)
#undef SWDFT_DCASE
  return hipErrorInvalidValue;
}

}  // namespace dense
}  // namespace swdft
