// Direct 2D SWDFT in FP64 (Eq. (2) evaluated literally): the comparator the
// tree is measured against, and the path for FP64 input.
//
// Every output coefficient is its own double sum over the n0 x n1 window,
//   y = s * sum_{j0} Omega0[j0 k0 mod n0] * ( sum_{j1} x[q0+j0][q1+j1] Omega1[j1 k1 mod n1] ),
// i.e. n0*n1 complex multiply-adds per coefficient with nothing shared
// between coefficients or windows (the O(P0 P1 n0^2 n1^2) cost of Sec. 4.1).
//
// A 256-thread block owns WB consecutive windows of one row q0: it stages the
// n0 x (WB + n1 - 1) input tile and both twiddle tables in LDS, then each
// thread produces coefficients t = (w, k0, k1) in output order, so the 16-byte
// complex128 stores of a wave are contiguous.
#include "internal.h"

namespace swdft {
namespace {

constexpr int kDirectThreads = 256;
constexpr int kDirectTileElems = 2048;  // LDS budget for the input tile (elements)

__host__ __device__ constexpr int direct_windows_per_block(int n0, int n1) {
  // enough coefficients for every thread, tile within the LDS budget (one
  // window's n0 x n1 tile always; 64 KiB at n0 = n1 = 64)
  int wb = 1;
  while (wb < 64 && wb * n0 * n1 < 8 * kDirectThreads &&
         n0 * (2 * wb + n1 - 1) <= kDirectTileElems)
    wb *= 2;
  return wb;
}

// LDS of one block: the n0 x (wb + n1 - 1) input tile, then both twiddle
// vectors.
__host__ __device__ constexpr int direct_tile_elems(int n0, int n1, int wb) {
  return n0 * (wb + n1 - 1);
}

// POW2: both sides are powers of two and (j k) mod n is a mask; otherwise it
// is stepped (e += k, minus n on overflow) for any n.
template <bool REAL, bool POW2>
__global__ __launch_bounds__(kDirectThreads) void direct_f64_kernel(const void* __restrict__ xv,
                                                                    double2* __restrict__ y,
                                                                    DirectGeom g, TwiddlesF64 tw,
                                                                    int wb) {
  extern __shared__ double2 lds[];
  const int n0 = g.n0, n1 = g.n1;
  double2* xs = lds;
  double2* w0s = lds + direct_tile_elems(n0, n1, wb);
  double2* w1s = w0s + n0;

  int id = blockIdx.x;
  const int tile1 = id % g.ntiles1;
  id /= g.ntiles1;
  const int64_t q0 = id % g.P0;
  const int b = (int)(id / g.P0);
  const int64_t q1_0 = (int64_t)tile1 * wb;
  const int64_t nwin = min((int64_t)wb, g.P1 - q1_0);
  const int cols = (int)nwin + n1 - 1;

  if (threadIdx.x < n0) w0s[threadIdx.x] = tw.w0[threadIdx.x];
  if (threadIdx.x < n1) w1s[threadIdx.x] = tw.w1[threadIdx.x];
  for (int e = threadIdx.x; e < n0 * cols; e += kDirectThreads) {
    const int j0 = e / cols, c = e % cols;
    const int64_t off = b * g.x_image_stride + (q0 + j0) * g.N1 + q1_0 + c;
    if constexpr (REAL) {
      xs[e] = make_double2(reinterpret_cast<const double*>(xv)[off], 0.0);
    } else {
      xs[e] = reinterpret_cast<const double2*>(xv)[off];
    }
  }
  __syncthreads();

  const int per_win = n0 * n1;
  const int total = (int)nwin * per_win;
  double2* ytile = y + b * g.y_image_stride + (q0 * g.P1 + q1_0) * per_win;
  for (int t = threadIdx.x; t < total; t += kDirectThreads) {
    const int w = t / per_win;
    const int k0 = (t / n1) % n0;
    const int k1 = t % n1;
    double ar = 0.0, ai = 0.0;
    int e0 = 0;  // (j0 k0) mod n0
    for (int j0 = 0; j0 < n0; ++j0) {
      const double2* xrow = xs + j0 * cols + w;
      double sr = 0.0, si = 0.0;
      int e1 = 0;  // (j1 k1) mod n1
      for (int j1 = 0; j1 < n1; ++j1) {
        double2 tw1;
        if constexpr (POW2) {
          tw1 = w1s[(j1 * k1) & (n1 - 1)];
        } else {
          tw1 = w1s[e1];
          e1 += k1;
          if (e1 >= n1) e1 -= n1;
        }
        const double2 v = xrow[j1];
        if constexpr (REAL) {
          sr += v.x * tw1.x;
          si += v.x * tw1.y;
        } else {
          sr += v.x * tw1.x - v.y * tw1.y;
          si += v.x * tw1.y + v.y * tw1.x;
        }
      }
      double2 tw0;
      if constexpr (POW2) {
        tw0 = w0s[(j0 * k0) & (n0 - 1)];
      } else {
        tw0 = w0s[e0];
        e0 += k0;
        if (e0 >= n0) e0 -= n0;
      }
      ar += tw0.x * sr - tw0.y * si;
      ai += tw0.x * si + tw0.y * sr;
    }
    ytile[t] = make_double2(ar * g.scale, ai * g.scale);
  }
}

}  // namespace

int direct_f64_windows_per_block(int n0, int n1) { return direct_windows_per_block(n0, n1); }

hipError_t launch_direct_f64(int n0, int n1, bool real_input, const void* x, double2* y,
                             const DirectGeom& g, const TwiddlesF64& tw, hipStream_t stream) {
  const int wb = direct_windows_per_block(n0, n1);
  const int64_t nb = (int64_t)g.batch * g.P0 * g.ntiles1;
  if (nb > 0x7fffffff) return hipErrorInvalidConfiguration;
  const size_t lds = (size_t)(direct_tile_elems(n0, n1, wb) + n0 + n1) * sizeof(double2);
  const bool pow2 = (n0 & (n0 - 1)) == 0 && (n1 & (n1 - 1)) == 0;
  const dim3 grid((unsigned)nb), block(kDirectThreads);
  if (real_input) {
    if (pow2) {
      hipLaunchKernelGGL((direct_f64_kernel<true, true>), grid, block, lds, stream, x, y, g, tw, wb);
    } else {
      hipLaunchKernelGGL((direct_f64_kernel<true, false>), grid, block, lds, stream, x, y, g, tw, wb);
    }
  } else {
    if (pow2) {
      hipLaunchKernelGGL((direct_f64_kernel<false, true>), grid, block, lds, stream, x, y, g, tw, wb);
    } else {
      hipLaunchKernelGGL((direct_f64_kernel<false, false>), grid, block, lds, stream, x, y, g, tw,
                         wb);
    }
  }
  return hipGetLastError();
}

}  // namespace swdft
