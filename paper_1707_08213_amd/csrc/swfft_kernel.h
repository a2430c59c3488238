// Per-window 2D FFT for gfx950: the 2D SWFFT that the tree is compared with
// (Sec. 4.1 and Table 1; the middle curve of Fig. 4). Every window's n0 x n1
// DFT is computed from scratch by a radix-2 row-column FFT (decimation in
// time), with nothing shared between windows: (n0 n1 / 2) log2(n0 n1)
// butterflies per window, O(P0 P1 n0 n1 log(n0 n1)) in total, against the
// tree's 2(n0 n1 - 1) node operations per window (Eq. (8)).
//
// The butterflies are those of the tree: a radix-2 DIT stage combines the
// sub-DFT of the even samples E and of the odd samples O of a segment as
// E + W^i O and E - W^i O, and in the tree's notation E is the level-(t-1)
// node of the earlier position p - s_t and O that of position p (Eq. (5),
// Eq. (6)). Rows go first, then columns, as in the tree, so both compute the
// same intermediate values (Sec. 4.6); they differ in how often each value is
// computed, not in what it is.
//
// Mapping: a 64-lane workgroup owns WW = 64 / max(n0, n1) consecutive windows
// of one window row at a time and walks RS window rows. Per row it stages the
// n0 x (WW + n1 - 1) input tile in LDS (coalesced loads), then lane (w, i)
//  1. for i < n0: runs the n1-point FFT of row i of window w and leaves it in
//     LDS, Z[w][i][k1];
//  2. for i < n1: runs the n0-point FFT of column k1 = i of Z[w] and stores
//     y[q0][q1_w][k0][k1] for every k0 (non-temporal from n1 = 16 on, where
//     a store covers whole 128-byte lines).
#pragma once

#include "tree_fwd_kernel.h"

namespace swdft {
namespace swfft {

using tree::cadd;
using tree::csub;
using tree::ilog2;
using tree::sfor;
using tree::twmul;

constexpr int bitrev(int v, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1) << (bits - 1 - b);
  return r;
}

// In-place N-point DFT of v (natural order in and out), radix-2 decimation
// in time: the input is permuted to bit-reversed order (register renaming
// only), then stage t = 1..log2 N combines blocks of 2^(t-1) into blocks of
// 2^t with twiddles w[i * N / 2^t].
template <int N>
__device__ __forceinline__ void fft_dit(float2 (&v)[N], const float2* w) {
  constexpr int M = ilog2(N);
  float2 a[N];
  sfor<0, N>([&](auto K) { a[K] = v[bitrev(K, M)]; });
  sfor<1, M + 1>([&](auto T) {
    constexpr int len = 1 << T;
    constexpr int h = len / 2;
    constexpr int s = N / len;
    sfor<0, N / len>([&](auto G) {
      sfor<0, h>([&](auto I) {
        constexpr int e = G * len + I;
        const float2 b = a[e];
        const float2 t = twmul<I * s, N>(a[e + h], w);
        a[e] = cadd(b, t);
        a[e + h] = csub(b, t);
      });
    });
  });
  sfor<0, N>([&](auto K) { v[K] = a[K]; });
}

template <int N0W, int N1W, bool REAL>
struct FftCfg {
  static constexpr int NM = N0W > N1W ? N0W : N1W;
  static constexpr int WW = 64 / NM;           // windows per workgroup and row
  static constexpr int TC = WW + N1W - 1;      // input tile columns
  static constexpr int XE = REAL ? 1 : 2;      // floats per input element
  static constexpr int ZS = N1W + 1;           // padded row of Z in LDS (float2)
  static constexpr int X_FLOATS = N0W * TC * XE;
  static constexpr int Z_FLOATS = WW * N0W * ZS * 2;
  static constexpr int LDS_FLOATS = X_FLOATS > Z_FLOATS ? X_FLOATS : Z_FLOATS;
};

template <int N0W, int N1W, bool REAL>
__global__ __launch_bounds__(64) void swfft_kernel(const void* __restrict__ xv,
                                                   float2* __restrict__ y, SwfftGeom g_in,
                                                   TwiddlesF32 tw) {
  using C = FftCfg<N0W, N1W, REAL>;
  __shared__ float lds[C::LDS_FLOATS];
  const SwfftGeom g = tree::uniform_copy(g_in);
  const int lane = threadIdx.x;
  int id = blockIdx.x;
  const int grp = id % g.ngroups;
  id /= g.ngroups;
  const int slab = id % g.nslabs;
  const int b = id / g.nslabs;
  const int64_t q1_0 = (int64_t)grp * C::WW;
  const int64_t q0_begin = (int64_t)slab * g.RS;
  const int64_t q0_end = min(q0_begin + (int64_t)g.RS, g.P0);

  const int w = lane / C::NM;
  const int i = lane % C::NM;
  const int64_t q1 = q1_0 + w;
  const bool win_ok = q1 < g.P1;

  using XT = std::conditional_t<REAL, float, float2>;
  const XT* ximg = reinterpret_cast<const XT*>(xv) + b * g.x_image_stride;
  float2* yimg = y + b * g.y_image_stride;
  XT* xs = reinterpret_cast<XT*>(lds);
  float2* zs = reinterpret_cast<float2*>(lds);

  for (int64_t q0 = q0_begin; q0 < q0_end; ++q0) {
    // input tile: rows q0 .. q0 + n0 - 1 (inside the image for every q0 <
    // P0), columns q1_0 .. q1_0 + TC - 1 (zero past the right edge)
    for (int e = lane; e < N0W * C::TC; e += 64) {
      const int r = e / C::TC, c = e % C::TC;
      const int64_t col = q1_0 + c;
      XT v{};
      if (col < g.N1) v = ximg[(q0 + r) * g.N1 + col];
      xs[e] = v;
    }
    __syncthreads();

    // 1. row FFTs (Eq. (5) levels): lane (w, i) takes row i of window w
    float2 v[N1W];
    if (i < N0W) {
      sfor<0, N1W>([&](auto J) {
        if constexpr (REAL) {
          v[J] = make_float2(xs[i * C::TC + w + J], 0.f);
        } else {
          v[J] = xs[i * C::TC + w + J];
        }
      });
      fft_dit<N1W>(v, tw.w1);
      if (g.scale != 1.0f) {
        sfor<0, N1W>([&](auto K) { v[K] = make_float2(v[K].x * g.scale, v[K].y * g.scale); });
      }
    }
    __syncthreads();  // the tile is read; its LDS now takes Z
    if (i < N0W) {
      float2* zrow = zs + (w * N0W + i) * C::ZS;
      sfor<0, N1W>([&](auto K) { zrow[K] = v[K]; });
    }
    __syncthreads();

    // 2. column FFTs (Eq. (6) levels): lane (w, i) takes column k1 = i
    if (i < N1W) {
      float2 u[N0W];
      const float2* zcol = zs + w * N0W * C::ZS + i;
      sfor<0, N0W>([&](auto J) { u[J] = zcol[J * C::ZS]; });
      fft_dit<N0W>(u, tw.w0);
      if (win_ok) {
        // non-temporal where a store covers whole 128-byte lines of a window
        float2* dst = yimg + ((q0 * g.P1 + q1) * N0W) * N1W + i;
        sfor<0, N0W>([&](auto K) {
          if constexpr (N1W >= 16) {
            tree::store_nt(dst + K * N1W, u[K]);
          } else {
            dst[K * N1W] = u[K];
          }
        });
      }
    }
    __syncthreads();  // Z is read before the next row's tile overwrites it
  }
}

template <int N0W, int N1W, bool REAL>
hipError_t launch_one(const void* x, float2* y, const SwfftGeom& g, const TwiddlesF32& tw,
                      hipStream_t stream) {
  const int64_t nb = (int64_t)g.batch * g.nslabs * g.ngroups;
  if (nb < 1 || nb > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((swfft_kernel<N0W, N1W, REAL>), dim3((unsigned)nb), dim3(64), 0, stream, x,
                     y, g, tw);
  return hipGetLastError();
}

template <int N0W, bool REAL>
hipError_t launch_n0(int n1, const void* x, float2* y, const SwfftGeom& g, const TwiddlesF32& tw,
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

template <bool REAL>
hipError_t launch(int n0, int n1, const void* x, float2* y, const SwfftGeom& g,
                  const TwiddlesF32& tw, hipStream_t s) {
  switch (n0) {
    case 1: return launch_n0<1, REAL>(n1, x, y, g, tw, s);
    case 2: return launch_n0<2, REAL>(n1, x, y, g, tw, s);
    case 4: return launch_n0<4, REAL>(n1, x, y, g, tw, s);
    case 8: return launch_n0<8, REAL>(n1, x, y, g, tw, s);
    case 16: return launch_n0<16, REAL>(n1, x, y, g, tw, s);
    case 32: return launch_n0<32, REAL>(n1, x, y, g, tw, s);
    case 64: return launch_n0<64, REAL>(n1, x, y, g, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace swfft

hipError_t launch_swfft_r(int n0, int n1, const void* x, float2* y, const SwfftGeom& g,
                          const TwiddlesF32& tw, hipStream_t s);
hipError_t launch_swfft_c(int n0, int n1, const void* x, float2* y, const SwfftGeom& g,
                          const TwiddlesF32& tw, hipStream_t s);

}  // namespace swdft
