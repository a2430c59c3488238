// swdft2d_backward_noalloc: the adjoint with its workspace in a fixed
// per-device array of the library instead of a plan-owned allocation, for
// callers that cannot allocate device memory (code under stream capture,
// tight serving loops). It runs the kernels of swdft2d_backward with the
// same launch shape, so its dx is bitwise that of swdft2d_backward.
#include <mutex>

#include "plan.h"

namespace {

constexpr size_t kScratchBytes = SWDFT_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch keeps 256-byte alignment");

// The workspace of every swdft2d_backward_noalloc call on a device. Each
// device that loads the library holds its own copy until the process ends.
// Host code never uses this name as an address: the device address comes
// from hipGetSymbolAddress, once per device (scratch_on).
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up on the
// first call on that device.
swdft_status_t scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return swdft::host::fail(SWDFT_E_DEVICE, "device %d out of range for the scratch table", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return swdft::host::device_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                      "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SWDFT_OK;
}

}  // namespace

extern "C" swdft_status_t swdft2d_backward_noalloc(swdft2d_plan_t plan, const void* dy, void* dx,
                                                   hipStream_t stream) {
  swdft::AdjGeom g{};
  size_t ws_bytes = 0;
  swdft_status_t st = swdft::host::backward_prepare(plan, dy, dx, &g, &ws_bytes);
  if (st != SWDFT_OK) return st;
  if (ws_bytes > kScratchBytes)
    return swdft::host::fail(SWDFT_E_NOMEM,
                             "the adjoint needs %zu bytes of workspace; the scratch array of "
                             "swdft2d_backward_noalloc holds %zu (use swdft2d_backward)",
                             ws_bytes, kScratchBytes);
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return swdft::host::device_fail(e, "hipGetDevice");
  void* ws = nullptr;
  st = scratch_on(dev, &ws);
  if (st != SWDFT_OK) return st;
  return swdft::host::backward_launch(plan, dy, ws, dx, g, stream);
}
