// C ABI of the streaming 2D sliding-window DFT (the real-time order of
// Sec. 4.3): rows arrive in calls of any size, the column-level state of the
// trees stays resident on the device, and every call emits the window rows
// its rows complete.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <unordered_set>

#include "plan.h"

struct swdft2d_stream_s {
  int64_t N1 = 0, P1 = 0;
  int32_t n0 = 0, n1 = 0;
  swdft_dtype_t dtype = SWDFT_R32;
  swdft_norm_t norm = SWDFT_NORM_NONE;
  swdft::TwiddlesF32 tw{};
  int64_t rows = 0;            // rows received so far (enqueued)
  float2* state = nullptr;     // resident ring state, allocated at the first push
  int64_t state_elems = 0;
  int device = -1;             // device holding the state
};

namespace swdft {
namespace host {
namespace {

std::mutex g_streams_mutex;

std::unordered_set<swdft2d_stream_s*>& live_streams() {
  static std::unordered_set<swdft2d_stream_s*> s;
  return s;
}

bool is_live_stream(swdft2d_stream_t s) {
  std::lock_guard<std::mutex> lk(g_streams_mutex);
  return s != nullptr && live_streams().count(s) != 0;
}

int64_t stream_nstrips(const swdft2d_stream_s* s) {
  return ceil_div(s->P1, swdft::tree_fwd_columns_per_wave(s->n0, s->n1,
                                                         swdft::tree_stream_kg(s->n0)));
}

// Window rows that complete when `rows` rows follow `before` rows: every window
// whose last row (q0 + n0 - 1) is among them.
int64_t completed(int64_t before, int64_t rows, int n0) {
  const int64_t lo = std::max<int64_t>(0, before - n0 + 1);
  const int64_t hi = std::max<int64_t>(0, before + rows - n0 + 1);
  return hi - lo;
}

// Allocate (first call) and clear the resident state on the current device.
swdft_status_t ensure_state(swdft2d_stream_s* s, hipStream_t stream) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (s->state) {
    if (dev != s->device)
      return fail(SWDFT_E_ARG, "the stream's state lives on device %d, not the current device %d",
                  s->device, dev);
    return SWDFT_OK;
  }
  const int64_t elems = (int64_t)swdft::tree_stream_state_slots(s->n0) * stream_nstrips(s) * 64;
  void* p = nullptr;
  e = hipMalloc(&p, (size_t)elems * sizeof(float2));
  if (e != hipSuccess) return fail(SWDFT_E_NOMEM, "stream state of %lld bytes: %s",
                                   (long long)(elems * 8), hipGetErrorString(e));
  s->state = static_cast<float2*>(p);
  s->state_elems = elems;
  s->device = dev;
  e = swdft::launch_fill_zero(s->state, elems, stream);
  if (e != hipSuccess) return device_fail(e, "stream state clear");
  return SWDFT_OK;
}

}  // namespace
}  // namespace host
}  // namespace swdft

using namespace swdft::host;

extern "C" {

swdft_status_t swdft2d_stream_create(swdft2d_stream_t* out, int64_t N1, int32_t n0, int32_t n1,
                                     swdft_dtype_t dtype) {
  if (!out) return fail(SWDFT_E_ARG, "stream output pointer is null");
  *out = nullptr;
  if (N1 < 1 || n0 < 1 || n1 < 1)
    return fail(SWDFT_E_ARG, "sizes must be >= 1 (N1=%lld, n=%d x %d)", (long long)N1, n0, n1);
  if ((int)dtype < (int)SWDFT_R32 || (int)dtype > (int)SWDFT_C64)
    return fail(SWDFT_E_ARG, "unknown dtype %d", (int)dtype);
  if (f64_dtype(dtype)) return fail(SWDFT_E_DTYPE, "streams take R32 or C32 input");
  if (!is_pow2(n0) || !is_pow2(n1))
    return fail(SWDFT_E_NOT_POW2, "window %d x %d is not radix-2", n0, n1);
  if (n1 > N1) return fail(SWDFT_E_WINDOW, "window width %d larger than the row length %lld", n1,
                           (long long)N1);
  if (n0 > SWDFT_MAX_WINDOW_ADJ || n1 > SWDFT_MAX_WINDOW_ADJ)
    return fail(SWDFT_E_WINDOW, "window %d x %d above the streams' maximum %d", n0, n1,
                SWDFT_MAX_WINDOW_ADJ);
  if (N1 > SWDFT_MAX_ROW)
    return fail(SWDFT_E_OVERFLOW, "row length %lld above the supported maximum %d",
                (long long)N1, SWDFT_MAX_ROW);
  auto* s = new (std::nothrow) swdft2d_stream_s();
  if (!s) return fail(SWDFT_E_NOMEM, "host allocation of the stream failed");
  s->N1 = N1;
  s->P1 = N1 - n1 + 1;
  s->n0 = n0;
  s->n1 = n1;
  s->dtype = dtype;
  make_twiddles_f32(n0, s->tw.w0);
  make_twiddles_f32(n1, s->tw.w1);
  {
    std::lock_guard<std::mutex> lk(g_streams_mutex);
    live_streams().insert(s);
  }
  *out = s;
  return SWDFT_OK;
}

swdft_status_t swdft2d_stream_set_norm(swdft2d_stream_t s, swdft_norm_t norm) {
  if (!is_live_stream(s)) return fail(SWDFT_E_PLAN, "null or destroyed stream");
  if (norm != SWDFT_NORM_NONE && norm != SWDFT_NORM_ORTHO)
    return fail(SWDFT_E_ARG, "unknown norm %d", (int)norm);
  s->norm = norm;
  return SWDFT_OK;
}

int64_t swdft2d_stream_rows(swdft2d_stream_t s) {
  if (!is_live_stream(s)) return -1;
  return s->rows;
}

int64_t swdft2d_stream_completes(swdft2d_stream_t s, int64_t rows) {
  if (!is_live_stream(s) || rows < 0) return -1;
  return completed(s->rows, rows, s->n0);
}

swdft_status_t swdft2d_stream_push(swdft2d_stream_t s, const void* x, int64_t rows, void* y,
                                   hipStream_t stream) {
  if (!is_live_stream(s)) return fail(SWDFT_E_PLAN, "null or destroyed stream");
  if (rows < 0) return fail(SWDFT_E_ARG, "negative row count");
  if (rows == 0) return SWDFT_OK;
  const int64_t nout = completed(s->rows, rows, s->n0);
  if (!x) return fail(SWDFT_E_ARG, "x is null");
  if (nout > 0 && !y) return fail(SWDFT_E_ARG, "y is null");
  const int64_t xe = x_elem_bytes(s->dtype);
  if ((uintptr_t)x % (uintptr_t)xe)
    return fail(SWDFT_E_ALIGN, "x is not %lld-byte aligned", (long long)xe);
  if (y && (uintptr_t)y % 8u) return fail(SWDFT_E_ALIGN, "y is not 8-byte aligned");
  int64_t xb = 0, yb = 0;
  if (!mul_ok(rows, s->N1 * xe, &xb) || !mul_ok(nout, s->P1 * s->n0 * s->n1 * 8, &yb))
    return fail(SWDFT_E_OVERFLOW, "push of %lld rows overflows", (long long)rows);
  if (y && ranges_overlap(x, xb, y, yb)) return fail(SWDFT_E_ARG, "x and y overlap");
  swdft_status_t st = ensure_state(s, stream);
  if (st != SWDFT_OK) return st;
  swdft::StreamGeom g{};
  g.N1 = s->N1;
  g.P1 = s->P1;
  g.rows_before = s->rows;
  g.rows = rows;
  g.nstrips = (int32_t)stream_nstrips(s);
  g.scale = norm_scale(s->norm, s->n0, s->n1);
  hipError_t e = swdft::launch_tree_stream(s->n0, s->n1, real_dtype(s->dtype), x,
                                           static_cast<float2*>(y), s->state, g, s->tw, stream);
  if (e != hipSuccess) return device_fail(e, "stream launch");
  s->rows += rows;
  return SWDFT_OK;
}

swdft_status_t swdft2d_stream_reset(swdft2d_stream_t s, hipStream_t stream) {
  if (!is_live_stream(s)) return fail(SWDFT_E_PLAN, "null or destroyed stream");
  s->rows = 0;
  if (s->state) {
    hipError_t e = swdft::launch_fill_zero(s->state, s->state_elems, stream);
    if (e != hipSuccess) return device_fail(e, "stream state clear");
  }
  return SWDFT_OK;
}

swdft_status_t swdft2d_stream_destroy(swdft2d_stream_t s) {
  if (s == nullptr) return SWDFT_OK;
  {
    std::lock_guard<std::mutex> lk(g_streams_mutex);
    auto it = live_streams().find(s);
    if (it == live_streams().end()) return fail(SWDFT_E_PLAN, "stream already destroyed or unknown");
    live_streams().erase(it);
  }
  swdft_status_t st = SWDFT_OK;
  if (s->state) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (s->device >= 0) (void)hipSetDevice(s->device);
    hipError_t e = hipFree(s->state);
    if (cur >= 0) (void)hipSetDevice(cur);
    if (e != hipSuccess) st = device_fail(e, "stream state free");
  }
  delete s;
  return st;
}

}  // extern "C"
