// Persistent class kernels of batched plans (see batched.h).
#pragma once

#include "batched.h"
#include "dense_mfma_kernel.h"
#include "tree_fwd_kernel.h"

namespace swdft {
namespace batched {

// Next work item of the wave (wave-uniform), or a value >= count when done.
__device__ __forceinline__ int next_item(unsigned* counter) {
  unsigned mine = 0;
  if (threadIdx.x == 0) mine = atomicAdd(counter, 1u);
  return __builtin_amdgcn_readfirstlane((int)mine);
}

template <int N0W, int N1W, bool REAL>
__global__ __launch_bounds__(64) void tree_class_kernel(BatchArgs a) {
  constexpr int KG = batched_kg(N0W, N1W);
  using C = tree::TreeCfg<N0W, N1W, REAL, KG>;
  __shared__ float2 zl[C::LDS_FLOAT2];
  for (int it = next_item(a.counter); it < a.count; it = next_item(a.counter)) {
    const BatchItem w = a.items[it];
    const int image = __builtin_amdgcn_readfirstlane(w.image);
    const int strip = __builtin_amdgcn_readfirstlane(w.strip);
    const int slab = __builtin_amdgcn_readfirstlane(w.slab);
    const BatchImage* im = a.images + image;
    const int64_t xo = tree::uniform_copy(im->x_offset);
    const int64_t yo = tree::uniform_copy(im->y_offset);
    const void* xi = REAL ? static_cast<const void*>(static_cast<const float*>(a.x) + xo)
                          : static_cast<const void*>(static_cast<const float2*>(a.x) + xo);
    tree::tree_fwd_tile<N0W, N1W, REAL, KG>(xi, a.y + yo, im->tree, a.tw.w0, a.tw.w1, strip, slab,
                                            0, zl);
    __syncthreads();
  }
}

template <int N0W, int N1W, bool REAL>
__global__ __launch_bounds__(64) void dense_class_kernel(BatchArgs a) {
  using C = dense::DenseCfg<N0W, N1W, REAL>;
  __shared__ __attribute__((aligned(16))) __bf16 zr[C::LDS_BF16];
  for (int it = next_item(a.counter); it < a.count; it = next_item(a.counter)) {
    const BatchItem w = a.items[it];
    const int image = __builtin_amdgcn_readfirstlane(w.image);
    const int strip = __builtin_amdgcn_readfirstlane(w.strip);
    const int slab = __builtin_amdgcn_readfirstlane(w.slab);
    const BatchImage* im = a.images + image;
    const int64_t xo = tree::uniform_copy(im->x_offset);
    const int64_t yo = tree::uniform_copy(im->y_offset);
    const void* xi = REAL ? static_cast<const void*>(static_cast<const float*>(a.x) + xo)
                          : static_cast<const void*>(static_cast<const float2*>(a.x) + xo);
    dense::dense_fwd_tile<N0W, N1W, REAL>(xi, a.y + yo, im->dense, a.tw.w0, a.tw.w1, strip, slab,
                                          0, zr);
    __syncthreads();
  }
}

template <bool REAL, bool DENSE>
const void* class_symbol(int n0, int n1) {
#define SWDFT_SYM(A, B)                                                          \
  if (n0 == A && n1 == B) {                                                      \
    if constexpr (DENSE)                                                         \
      return reinterpret_cast<const void*>(&dense_class_kernel<A, B, REAL>);     \
    else                                                                         \
      return reinterpret_cast<const void*>(&tree_class_kernel<A, B, REAL>);      \
  }
  SWDFT_SYM(8, 8)
  SWDFT_SYM(8, 16)
  SWDFT_SYM(8, 32)
  SWDFT_SYM(16, 8)
  SWDFT_SYM(16, 16)
  SWDFT_SYM(16, 32)
  SWDFT_SYM(32, 8)
  SWDFT_SYM(32, 16)
  SWDFT_SYM(32, 32)
#undef SWDFT_SYM
  return nullptr;
}

}  // namespace batched
}  // namespace swdft
