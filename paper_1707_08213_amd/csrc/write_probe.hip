// Measurement aid: fill a buffer with a constant at the device's HBM write
// ceiling, for comparison with the tree's output stream.
#include <cstdint>

#include "internal.h"

namespace swdft {

namespace {

// The access pattern of a device memset: 256 workgroups of 256 lanes, each
// lane storing 16 bytes per step, the grid sweeping the buffer front to back.
// A head element aligns the 16-byte stores; an odd tail element is stored
// alone.
constexpr int kProbeBlocks = 256;
constexpr int kProbeThreads = 256;

__global__ __launch_bounds__(kProbeThreads) void write_probe_kernel(float2* __restrict__ y,
                                                                    int64_t n) {
  const float2 v = make_float2(1.0f, -1.0f);
  const bool first = blockIdx.x == 0 && threadIdx.x == 0;
  const int64_t head = ((reinterpret_cast<uintptr_t>(y) & 15u) != 0 && n > 0) ? 1 : 0;
  if (head && first) y[0] = v;
  const int64_t n4 = (n - head) / 2;
  float4* y4 = reinterpret_cast<float4*>(y + head);
  const float4 v4 = make_float4(v.x, v.y, v.x, v.y);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) y4[i] = v4;
  if (first && head + 2 * n4 < n) y[n - 1] = v;
}

}  // namespace

hipError_t launch_write_probe(float2* y, int64_t n_float2, hipStream_t stream) {
  hipLaunchKernelGGL(write_probe_kernel, dim3(kProbeBlocks), dim3(kProbeThreads), 0, stream, y,
                     n_float2);
  return hipGetLastError();
}

}  // namespace swdft
