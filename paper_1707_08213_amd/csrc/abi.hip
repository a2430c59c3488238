// Host side of libswdft2d: plan objects, argument validation, twiddle
// generation and kernel dispatch behind the C ABI of include/swdft2d.h.
//
// Plans are plain host objects. Nothing here touches the GPU until exec or
// backward enqueue work, so every validation path runs on a machine without
// a GPU.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>

#include "plan.h"

using swdft::TwiddlesF32;
using swdft::TwiddlesF64;

namespace swdft {
namespace host {

thread_local std::string g_last_error;

std::mutex g_plans_mutex;
std::unordered_set<swdft2d_plan_s*>& live_plans() {
  static std::unordered_set<swdft2d_plan_s*> s;
  return s;
}

swdft_status_t fail(swdft_status_t st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

swdft_status_t device_fail(hipError_t e, const char* what) {
  return fail(SWDFT_E_DEVICE, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

bool is_live(swdft2d_plan_t p) {
  std::lock_guard<std::mutex> lk(g_plans_mutex);
  return p != nullptr && live_plans().count(p) != 0;
}

void register_plan(swdft2d_plan_s* p) {
  std::lock_guard<std::mutex> lk(g_plans_mutex);
  live_plans().insert(p);
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

bool mul_ok(int64_t a, int64_t b, int64_t* out) {
  if (a < 0 || b < 0) return false;
  if (a != 0 && b > INT64_MAX / a) return false;
  *out = a * b;
  return true;
}

bool real_dtype(swdft_dtype_t d) { return d == SWDFT_R32 || d == SWDFT_R64; }
bool f64_dtype(swdft_dtype_t d) { return d == SWDFT_R64 || d == SWDFT_C64; }
int64_t x_elem_bytes(swdft_dtype_t d) {
  switch (d) {
    case SWDFT_R32: return 4;
    case SWDFT_C32: return 8;
    case SWDFT_R64: return 8;
    default: return 16;
  }
}
int64_t y_elem_bytes(swdft_dtype_t d) { return f64_dtype(d) ? 16 : 8; }

// Omega[m] = exp(-2 pi i m / n), m < n, in FP64. For even n the first half
// is evaluated with cos/sin except at the exact points m = 0 (1) and m = n/4
// (-i), and the second half is the exact negation Omega[m + n/2] = -Omega[m];
// odd n (the mixed-radix sides 3 and 9) are evaluated directly for every m.
void make_twiddles(int n, double2* w) {
  const double two_pi = 6.283185307179586476925286766559;
  if (n == 1) {
    w[0] = make_double2(1.0, 0.0);
    return;
  }
  const int half = n % 2 == 0 ? n / 2 : n;
  for (int m = 0; m < half; ++m) {
    if (m == 0) {
      w[m] = make_double2(1.0, 0.0);
    } else if (4 * m == n) {
      w[m] = make_double2(0.0, -1.0);
    } else {
      const double a = two_pi * (double)m / (double)n;
      w[m] = make_double2(std::cos(a), -std::sin(a));
    }
  }
  for (int m = half; m < n; ++m) w[m] = make_double2(-w[m - half].x, -w[m - half].y);
}

// FP64 twiddles rounded once (round to nearest even) to FP32.
void make_twiddles_f32(int n, float2* w) {
  double2 d[kMaxWindow];
  make_twiddles(n, d);
  for (int m = 0; m < n; ++m) w[m] = make_float2((float)d[m].x, (float)d[m].y);
}

float norm_scale(swdft_norm_t norm, int n0, int n1) {
  return norm == SWDFT_NORM_ORTHO ? (float)(1.0 / std::sqrt((double)n0 * n1)) : 1.0f;
}

swdft_algo_t resolve_algo(const swdft2d_plan_s* p) {
  if (p->algo != SWDFT_ALGO_AUTO) return p->algo;
  if (p->tuned_algo != SWDFT_ALGO_AUTO) return p->tuned_algo;
  return f64_dtype(p->dtype) ? SWDFT_ALGO_DIRECT_F64 : SWDFT_ALGO_TREE;
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// dx rows per wave of the adjoint: a whole image column when that already
// gives enough waves (no dy row is then read twice); otherwise slabs, each
// primed by the n0-1 window rows below it.
int32_t adj_kg(const swdft2d_plan_s* p) {
  const int kg = env_int("SWDFT_ADJ_KG", 0);
  return kg > 0 && swdft::tree_adj_kg_supported(p->n0, p->n1, kg)
             ? kg
             : swdft::tree_adj_default_kg(p->n0, p->n1);
}

int32_t adj_slab(const swdft2d_plan_s* p, int kg) {
  const int cr = swdft::tree_adj_rows_per_chunk(p->n0, p->n1, kg);
  const int64_t nstrips = ceil_div(p->P1, swdft::tree_adj_columns_per_wave(p->n0, p->n1, kg));
  const int64_t full = ceil_div(p->N0, cr) * cr;
  int64_t S = 0;
  const char* env = std::getenv("SWDFT_ADJ_SLAB");
  if (env) S = std::atoll(env);
  if (S <= 0) {
    // Whole columns once they give about 1.5 waves per CU; otherwise about
    // two per CU (512 waves): more, shorter slabs re-read more priming rows of
    // dy than their extra waves gain (2048x512 / 32x8: 4 slabs 381 us, 8 slabs
    // 392 us; 1024^2 / 16x16: 2 slabs 372 us, 4 slabs 375 us).
    const int64_t waves_full = nstrips * p->batch;
    if (waves_full >= 384) {
      S = full;
    } else {
      const int64_t slabs = std::max<int64_t>(1, (512 + waves_full / 2) / waves_full);
      S = std::max<int64_t>(ceil_div(p->N0, slabs), 8 * (int64_t)(p->n0 - 1));
    }
  }
  S = std::max<int64_t>(S, cr);
  S = ceil_div(S, cr) * cr;
  S = std::min<int64_t>(S, full);
  return (int32_t)S;
}

swdft::AdjGeom adj_geom(const swdft2d_plan_s* p) {
  swdft::AdjGeom g{};
  g.N0 = p->N0;
  g.N1 = p->N1;
  g.P0 = p->P0;
  g.P1 = p->P1;
  g.y_image_stride = p->P0 * p->P1 * p->n0 * p->n1;
  g.kg = adj_kg(p);
  g.S = adj_slab(p, g.kg);
  g.nstrips = (int32_t)ceil_div(p->P1, swdft::tree_adj_columns_per_wave(p->n0, p->n1, g.kg));
  g.nslabs = (int32_t)ceil_div(p->N0, g.S);
  g.batch = (int32_t)p->batch;
  g.scale = p->norm == SWDFT_NORM_ORTHO ? (float)(1.0 / std::sqrt((double)p->n0 * p->n1)) : 1.0f;
  // As many resident workgroups as fit. With four rows of dy in flight per
  // wave (n0 <= 16) no cap was faster (16 x 256^2 / 16 x 16: 346 us uncapped,
  // 367 us at two per CU); SWDFT_ADJ_WPC sets a cap.
  g.wpc = env_int("SWDFT_ADJ_WPC", 0);
  g.lds_cu = lds_per_cu();
  if (g.lds_cu <= 0 || g.wpc < 0) g.wpc = 0;
  return g;
}

// Make sure the plan's workspace holds `bytes` on the current device.
swdft_status_t ensure_workspace(swdft2d_plan_s* p, size_t bytes) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (p->workspace && p->workspace_device == dev && p->workspace_bytes >= bytes) return SWDFT_OK;
  if (p->workspace) {
    // the previous buffer may still be in use by work on another device/stream
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return device_fail(e, "hipDeviceSynchronize");
    int cur = dev;
    if (p->workspace_device >= 0 && p->workspace_device != dev) (void)hipSetDevice(p->workspace_device);
    (void)hipFree(p->workspace);
    if (cur != p->workspace_device) (void)hipSetDevice(cur);
    p->workspace = nullptr;
    p->workspace_bytes = 0;
  }
  void* ptr = nullptr;
  e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(SWDFT_E_NOMEM, "workspace of %zu bytes: %s", bytes, hipGetErrorString(e));
  }
  p->workspace = ptr;
  p->workspace_bytes = bytes;
  p->workspace_device = dev;
  return SWDFT_OK;
}

// Window rows per wave of the dense kernel: a multiple of 16 (one row chunk),
// enough waves to fill the chip, and long enough that the row products
// recomputed at each slab top (n0 - 1 rows, rounded to 16) stay small.
swdft::DenseGeom dense_geom(const swdft2d_plan_s* p) {
  swdft::DenseGeom g{};
  g.N0 = p->N0;
  g.N1 = p->N1;
  g.P0 = p->P0;
  g.P1 = p->P1;
  g.x_image_stride = p->N0 * p->N1;
  g.y_image_stride = p->P0 * p->P1 * p->n0 * p->n1;
  g.nstrips = (int32_t)ceil_div(p->P1, swdft::dense_columns_per_wave(p->n0, p->n1));
  int64_t S = p->dense_slab;
  if (S <= 0) {
    const char* env = std::getenv("SWDFT_DENSE_SLAB");
    if (env) S = std::atoll(env);
  }
  if (S <= 0) {
    // about 1024 tiles for windows of 256 values and up, 4096 below (sweep of
    // 512-4096 tiles on gfx950: 2048x512 / 32x8 437 -> 371 us, 1024^2 /
    // 16x16 394 -> 331 us, 8x32 423 -> 398 us, 512^2 / 16x16 102 -> 86 us;
    // 1024^2 / 8x8 111 -> 156 us, so small windows keep the 4096)
    const int64_t tiles = (int64_t)p->n0 * p->n1 >= 256 ? 1024 : 4096;
    S = ceil_div(p->P0 * g.nstrips * p->batch, tiles);
    S = std::max<int64_t>(S, 64);
  }
  S = ceil_div(std::max<int64_t>(S, 16), 16) * 16;
  S = std::min<int64_t>(S, ceil_div(p->P0, 16) * 16);
  g.S = (int32_t)S;
  g.nslabs = (int32_t)ceil_div(p->P0, g.S);
  g.batch = (int32_t)p->batch;
  g.scale = p->norm == SWDFT_NORM_ORTHO ? (float)(1.0 / std::sqrt((double)p->n0 * p->n1)) : 1.0f;
  return g;
}

swdft::DirectGeom direct_geom(const swdft2d_plan_s* p) {
  swdft::DirectGeom g{};
  g.N0 = p->N0;
  g.N1 = p->N1;
  g.P0 = p->P0;
  g.P1 = p->P1;
  g.x_image_stride = p->N0 * p->N1;
  g.y_image_stride = p->P0 * p->P1 * p->n0 * p->n1;
  g.n0 = p->n0;
  g.n1 = p->n1;
  g.ntiles1 = (int32_t)ceil_div(p->P1, swdft::direct_f64_windows_per_block(p->n0, p->n1));
  g.batch = (int32_t)p->batch;
  g.scale = p->norm == SWDFT_NORM_ORTHO ? 1.0 / std::sqrt((double)p->n0 * p->n1) : 1.0;
  return g;
}

// Window rows per workgroup of the per-window FFT: enough workgroups (about
// 8192) to fill the chip a few times over, each walking a run of rows.
swdft::SwfftGeom swfft_geom(const swdft2d_plan_s* p) {
  swdft::SwfftGeom g{};
  g.N0 = p->N0;
  g.N1 = p->N1;
  g.P0 = p->P0;
  g.P1 = p->P1;
  g.x_image_stride = p->N0 * p->N1;
  g.y_image_stride = p->P0 * p->P1 * p->n0 * p->n1;
  g.ngroups = (int32_t)ceil_div(p->P1, swdft::swfft_windows_per_group(p->n0, p->n1));
  const int64_t per_row = (int64_t)g.ngroups * p->batch;
  const int64_t nslabs = std::min<int64_t>(p->P0, std::max<int64_t>(1, ceil_div(8192, per_row)));
  g.RS = (int32_t)ceil_div(p->P0, nslabs);
  g.nslabs = (int32_t)ceil_div(p->P0, g.RS);
  g.batch = (int32_t)p->batch;
  g.scale = norm_scale(p->norm, p->n0, p->n1);
  return g;
}

bool ranges_overlap(const void* a, int64_t abytes, const void* b, int64_t bbytes) {
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + (uintptr_t)bbytes && b0 < a0 + (uintptr_t)abytes;
}

swdft_status_t check_buffers(const swdft2d_plan_s* p, const void* in, int64_t in_align,
                             int64_t in_bytes, const void* out, int64_t out_align,
                             int64_t out_bytes, const char* in_name, const char* out_name) {
  if (!in) return fail(SWDFT_E_ARG, "%s is null", in_name);
  if (!out) return fail(SWDFT_E_ARG, "%s is null", out_name);
  if ((uintptr_t)in % (uintptr_t)in_align)
    return fail(SWDFT_E_ALIGN, "%s is not %lld-byte aligned", in_name, (long long)in_align);
  if ((uintptr_t)out % (uintptr_t)out_align)
    return fail(SWDFT_E_ALIGN, "%s is not %lld-byte aligned", out_name, (long long)out_align);
  if (ranges_overlap(in, in_bytes, out, out_bytes))
    return fail(SWDFT_E_ARG, "%s and %s overlap", in_name, out_name);
  (void)p;
  return SWDFT_OK;
}

swdft_status_t backward_prepare(swdft2d_plan_t plan, const void* dy, void* dx, AdjGeom* g,
                                size_t* ws_bytes) {
  if (!is_live(plan)) return fail(SWDFT_E_PLAN, "null or destroyed plan");
  if (plan->kind == 1) return fail(SWDFT_E_PLAN, "backward is not available for batched plans");
  if (plan->n0 > SWDFT_MAX_WINDOW_ADJ || plan->n1 > SWDFT_MAX_WINDOW_ADJ || mixed_window(plan))
    return fail(SWDFT_E_WINDOW, "backward supports power-of-two windows up to %d, not %d x %d",
                SWDFT_MAX_WINDOW_ADJ, plan->n0, plan->n1);
  const swdft2d_plan_s* p = plan;
  const int64_t xb = p->batch * p->N0 * p->N1 * x_elem_bytes(p->dtype);
  const int64_t yb = swdft2d_output_bytes(plan);
  swdft_status_t st = check_buffers(p, dy, y_elem_bytes(p->dtype), yb, dx,
                                    x_elem_bytes(p->dtype), xb, "dy", "dx");
  if (st != SWDFT_OK) return st;
  // The adjoint is always the transposed tree, whichever forward kernel an
  // AUTO plan ends up running (the tuner may pick the dense variant for the
  // forward transform; the adjoint of the map x -> y is the same).
  if (f64_dtype(p->dtype) || (p->algo != SWDFT_ALGO_AUTO && p->algo != SWDFT_ALGO_TREE))
    return fail(SWDFT_E_DTYPE, "backward runs the transposed tree; it needs an R32/C32 plan "
                "with the TREE (or AUTO) algorithm");
  *g = adj_geom(p);
  *ws_bytes =
      (size_t)swdft::tree_adj_workspace_elems(p->n0, p->n1, *g) * (real_dtype(p->dtype) ? 4 : 8);
  return SWDFT_OK;
}

swdft_status_t backward_launch(const swdft2d_plan_s* p, const void* dy, void* ws, void* dx,
                               const AdjGeom& g, hipStream_t stream) {
  hipError_t e = swdft::launch_tree_adj(p->n0, p->n1, real_dtype(p->dtype),
                                        static_cast<const float2*>(dy), ws, dx, g, p->tw32,
                                        stream);
  if (e != hipSuccess) return device_fail(e, "adjoint launch");
  return SWDFT_OK;
}


}  // namespace host
}  // namespace swdft

using namespace swdft::host;

extern "C" {

swdft_status_t swdft2d_plan(swdft2d_plan_t* out, int64_t N0, int64_t N1, int32_t n0, int32_t n1,
                            swdft_dtype_t dtype, int64_t batch) {
  if (!out) return fail(SWDFT_E_ARG, "plan output pointer is null");
  *out = nullptr;
  if (N0 < 1 || N1 < 1 || n0 < 1 || n1 < 1 || batch < 1)
    return fail(SWDFT_E_ARG, "sizes must be >= 1 (N=%lld x %lld, n=%d x %d, batch=%lld)",
                (long long)N0, (long long)N1, n0, n1, (long long)batch);
  if ((int)dtype < (int)SWDFT_R32 || (int)dtype > (int)SWDFT_C64)
    return fail(SWDFT_E_ARG, "unknown dtype %d", (int)dtype);
  if ((!is_pow2(n0) || !is_pow2(n1)) && !swdft::tree_mixed_supported(n0, n1))
    return fail(SWDFT_E_NOT_POW2, "window %d x %d: sides must be powers of two, or from "
                "{3, 6, 9, 12, 24} paired with each other or with {4, 8, 16}", n0, n1);
  if (n0 > N0 || n1 > N1)
    return fail(SWDFT_E_WINDOW, "window %d x %d larger than array %lld x %lld", n0, n1,
                (long long)N0, (long long)N1);
  if (n0 > SWDFT_MAX_WINDOW || n1 > SWDFT_MAX_WINDOW)
    return fail(SWDFT_E_WINDOW, "window %d x %d above the supported maximum %d", n0, n1,
                SWDFT_MAX_WINDOW);
  const int64_t P0 = N0 - n0 + 1, P1 = N1 - n1 + 1;
  int64_t t = 0, elems = 0, bytes = 0, xel = 0, xbytes = 0;
  if (!mul_ok(P0, P1, &t) || !mul_ok(t, (int64_t)n0 * n1, &t) || !mul_ok(t, batch, &elems) ||
      !mul_ok(elems, y_elem_bytes(dtype), &bytes) || !mul_ok(N0, N1, &xel) ||
      !mul_ok(xel, batch, &xel) || !mul_ok(xel, x_elem_bytes(dtype), &xbytes))
    return fail(SWDFT_E_OVERFLOW, "output of %lld images of %lld x %lld with %d x %d windows "
                "overflows int64", (long long)batch, (long long)N0, (long long)N1, n0, n1);
  if (batch > INT32_MAX || P0 > INT32_MAX || P1 > INT32_MAX)
    return fail(SWDFT_E_OVERFLOW, "batch or window count above 2^31-1");
  if (N1 > SWDFT_MAX_ROW)
    return fail(SWDFT_E_OVERFLOW, "row length %lld above the supported maximum %d",
                (long long)N1, SWDFT_MAX_ROW);

  auto* p = new (std::nothrow) swdft2d_plan_s();
  if (!p) return fail(SWDFT_E_NOMEM, "host allocation of the plan failed");
  p->N0 = N0;
  p->N1 = N1;
  p->P0 = P0;
  p->P1 = P1;
  p->n0 = n0;
  p->n1 = n1;
  p->batch = batch;
  p->dtype = dtype;
  make_twiddles(n0, p->tw64.w0);
  make_twiddles(n1, p->tw64.w1);
  make_twiddles_f32(n0, p->tw32.w0);
  make_twiddles_f32(n1, p->tw32.w1);
  register_plan(p);
  *out = p;
  return SWDFT_OK;
}

swdft_status_t swdft2d_set_norm(swdft2d_plan_t plan, swdft_norm_t norm) {
  if (!is_live(plan)) return fail(SWDFT_E_PLAN, "null or destroyed plan");
  if (norm != SWDFT_NORM_NONE && norm != SWDFT_NORM_ORTHO)
    return fail(SWDFT_E_ARG, "unknown norm %d", (int)norm);
  plan->norm = norm;
  if (plan->bs) batched_build_tables(plan);
  return SWDFT_OK;
}

swdft_status_t swdft2d_set_algo(swdft2d_plan_t plan, swdft_algo_t algo) {
  if (!is_live(plan)) return fail(SWDFT_E_PLAN, "null or destroyed plan");
  if (plan->kind == 1) {
    if (algo != SWDFT_ALGO_AUTO && algo != SWDFT_ALGO_TREE && algo != SWDFT_ALGO_DENSE_BF16X2)
      return fail((int)algo == SWDFT_ALGO_DIRECT_F64 ? SWDFT_E_DTYPE : SWDFT_E_ARG,
                  "batched plans run the tree or the dense variant");
    plan->algo = algo;
    if (algo != SWDFT_ALGO_AUTO)
      for (auto& kv : plan->bs->cfg) kv.second.dense = (algo == SWDFT_ALGO_DENSE_BF16X2);
    batched_build_tables(plan);
    return SWDFT_OK;
  }
  switch (algo) {
    case SWDFT_ALGO_AUTO: break;
    case SWDFT_ALGO_TREE:
    case SWDFT_ALGO_DENSE_BF16X2:
    case SWDFT_ALGO_SWFFT:
      if (f64_dtype(plan->dtype))
        return fail(SWDFT_E_DTYPE, "algorithm %d computes in FP32 and needs an R32/C32 plan",
                    (int)algo);
      if (algo == SWDFT_ALGO_SWFFT && mixed_window(plan))
        return fail(SWDFT_E_WINDOW, "the per-window FFT is radix-2; window %d x %d is not",
                    plan->n0, plan->n1);
      if (algo == SWDFT_ALGO_DENSE_BF16X2 && !swdft::dense_supported(plan->n0, plan->n1))
        return fail(SWDFT_E_WINDOW, "the dense BF16x2 algorithm supports n0, n1 in {8, 16, 32}, "
                    "not %d x %d", plan->n0, plan->n1);
      break;
    case SWDFT_ALGO_DIRECT_F64:
      if (!f64_dtype(plan->dtype))
        return fail(SWDFT_E_DTYPE, "DIRECT_F64 needs an R64/C64 plan (widen FP32 input first)");
      break;
    default:
      return fail(SWDFT_E_ARG, "unknown algorithm %d", (int)algo);
  }
  plan->algo = algo;
  return SWDFT_OK;
}

swdft_status_t swdft2d_exec(swdft2d_plan_t plan, const void* x, void* y, hipStream_t stream) {
  if (!is_live(plan)) return fail(SWDFT_E_PLAN, "null or destroyed plan");
  if (plan->kind == 1) return batched_exec(plan, x, y, stream);
  if (!plan->tuned) apply_cached_tuning(plan);
  const swdft2d_plan_s* p = plan;
  const int64_t xb = p->batch * p->N0 * p->N1 * x_elem_bytes(p->dtype);
  const int64_t yb = swdft2d_output_bytes(plan);
  swdft_status_t st = check_buffers(p, x, x_elem_bytes(p->dtype), xb, y, y_elem_bytes(p->dtype),
                                    yb, "x", "y");
  if (st != SWDFT_OK) return st;
  hipError_t e = hipSuccess;
  switch (resolve_algo(p)) {
    case SWDFT_ALGO_TREE:
      if (mixed_window(p)) {
        e = real_dtype(p->dtype)
                ? swdft::launch_tree_mixed_r(p->n0, p->n1, x, static_cast<float2*>(y),
                                             tree_geom_cached(plan), p->tw32, stream)
                : swdft::launch_tree_mixed_c(p->n0, p->n1, x, static_cast<float2*>(y),
                                             tree_geom_cached(plan), p->tw32, stream);
      } else {
        e = swdft::launch_tree_fwd(p->n0, p->n1, real_dtype(p->dtype), x,
                                   static_cast<float2*>(y), tree_geom_cached(plan), p->tw32,
                                   stream);
      }
      break;
    case SWDFT_ALGO_DENSE_BF16X2:
      e = swdft::launch_dense_fwd(p->n0, p->n1, real_dtype(p->dtype), x, static_cast<float2*>(y),
                                  dense_geom(p), p->tw32, stream);
      break;
    case SWDFT_ALGO_SWFFT:
      e = swdft::launch_swfft(p->n0, p->n1, real_dtype(p->dtype), x, static_cast<float2*>(y),
                              swfft_geom(p), p->tw32, stream);
      break;
    case SWDFT_ALGO_DIRECT_F64:
      e = swdft::launch_direct_f64(p->n0, p->n1, real_dtype(p->dtype), x,
                                   static_cast<double2*>(y), direct_geom(p), p->tw64, stream);
      break;
    default:
      return fail(SWDFT_E_DTYPE, "algorithm not available for this plan");
  }
  if (e != hipSuccess) return device_fail(e, "forward launch");
  return SWDFT_OK;
}


swdft_status_t swdft2d_backward(swdft2d_plan_t plan, const void* dy, void* dx, hipStream_t stream) {
  swdft::AdjGeom g{};
  size_t ws_bytes = 0;
  swdft_status_t st = backward_prepare(plan, dy, dx, &g, &ws_bytes);
  if (st != SWDFT_OK) return st;
  st = ensure_workspace(plan, ws_bytes);
  if (st != SWDFT_OK) return st;
  return backward_launch(plan, dy, plan->workspace, dx, g, stream);
}

swdft_status_t swdft2d_twiddles(swdft2d_plan_t plan, int32_t axis, float* out, int32_t len) {
  if (!is_live(plan)) return fail(SWDFT_E_PLAN, "null or destroyed plan");
  if (plan->kind != 0) return fail(SWDFT_E_PLAN, "a batched plan has one twiddle table per shape");
  if (axis != 0 && axis != 1) return fail(SWDFT_E_ARG, "axis must be 0 or 1, not %d", axis);
  const int n = axis == 0 ? plan->n0 : plan->n1;
  if (out == nullptr || len < 2 * n)
    return fail(SWDFT_E_ARG, "twiddle output needs %d floats", 2 * n);
  const float2* w = axis == 0 ? plan->tw32.w0 : plan->tw32.w1;
  for (int m = 0; m < n; ++m) {
    out[2 * m] = w[m].x;
    out[2 * m + 1] = w[m].y;
  }
  return SWDFT_OK;
}

swdft_status_t swdft2d_destroy(swdft2d_plan_t plan) {
  if (plan == nullptr) return SWDFT_OK;
  {
    std::lock_guard<std::mutex> lk(g_plans_mutex);
    auto it = live_plans().find(plan);
    if (it == live_plans().end()) return fail(SWDFT_E_PLAN, "plan already destroyed or unknown");
    live_plans().erase(it);
  }
  swdft_status_t st = SWDFT_OK;
  if (plan->workspace) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (plan->workspace_device >= 0) (void)hipSetDevice(plan->workspace_device);
    hipError_t e = hipFree(plan->workspace);
    if (cur >= 0) (void)hipSetDevice(cur);
    if (e != hipSuccess) st = device_fail(e, "workspace free");
  }
  if (plan->bs) {
    batched_free(plan->bs);
    delete plan->bs;
  }
  delete plan;
  return st;
}

int64_t swdft2d_output_elems(swdft2d_plan_t plan) {
  if (!is_live(plan)) return -1;
  if (plan->kind == 1) return plan->bs->out_elems;
  return plan->batch * plan->P0 * plan->P1 * plan->n0 * plan->n1;
}

int64_t swdft2d_output_bytes(swdft2d_plan_t plan) {
  if (!is_live(plan)) return -1;
  return swdft2d_output_elems(plan) * y_elem_bytes(plan->dtype);
}

swdft_status_t swdft2d_describe(swdft2d_plan_t plan, char* buf, int32_t len) {
  if (!is_live(plan)) return fail(SWDFT_E_PLAN, "null or destroyed plan");
  if (!buf || len < 1) return fail(SWDFT_E_ARG, "describe buffer is null or empty");
  const swdft2d_plan_s* p = plan;
  if (p->kind == 1) {
    const swdft::BatchState* bs = p->bs;
    std::string d = "kind=batched images=" + std::to_string(bs->descs.size()) +
                    " items=" + std::to_string(bs->items.size()) + " classes=";
    for (const auto& c : bs->classes)
      d += std::to_string(c.n0) + "x" + std::to_string(c.n1) + (c.dense ? ":dense" : ":tree") +
           "/" + std::to_string(c.item_count) + " ";
    snprintf(buf, (size_t)len, "%s", d.c_str());
    return SWDFT_OK;
  }
  const swdft_algo_t a = resolve_algo(p);
  if (a == SWDFT_ALGO_TREE) {
    const swdft::TreeGeom g = tree_geom(p);
    snprintf(buf, (size_t)len,
             "algo=tree n=%dx%d N=%lldx%lld batch=%lld kg=%d cols_per_wave=%d rows_per_chunk=%d "
             "slab=%d strips=%d slabs=%d waves=%lld waves_per_strip=%d groups_per_cu=%d order=%s "
             "radix=%s",
             p->n0, p->n1, (long long)p->N0, (long long)p->N1, (long long)p->batch, g.kg,
             swdft::tree_fwd_columns_per_wave(p->n0, p->n1, g.kg), tree_chunk_rows(p, g.kg, g.wv),
             g.S, g.nstrips, g.nslabs, (long long)g.nstrips * g.nslabs * p->batch * g.wv, g.wv,
             g.wpc, g.order ? "dispatch" : "xcd", mixed_window(p) ? "2,3" : "2");
  } else if (a == SWDFT_ALGO_DENSE_BF16X2) {
    const swdft::DenseGeom g = dense_geom(p);
    snprintf(buf, (size_t)len,
             "algo=dense_bf16x2 n=%dx%d N=%lldx%lld batch=%lld cols_per_wave=%d slab=%d strips=%d "
             "slabs=%d waves=%lld",
             p->n0, p->n1, (long long)p->N0, (long long)p->N1, (long long)p->batch,
             swdft::dense_columns_per_wave(p->n0, p->n1), g.S, g.nstrips, g.nslabs,
             (long long)g.nstrips * g.nslabs * p->batch);
  } else if (a == SWDFT_ALGO_SWFFT) {
    const swdft::SwfftGeom g = swfft_geom(p);
    snprintf(buf, (size_t)len,
             "algo=swfft n=%dx%d N=%lldx%lld batch=%lld windows_per_group=%d rows_per_group=%d "
             "groups=%lld",
             p->n0, p->n1, (long long)p->N0, (long long)p->N1, (long long)p->batch,
             swdft::swfft_windows_per_group(p->n0, p->n1), g.RS,
             (long long)g.ngroups * g.nslabs * p->batch);
  } else {
    snprintf(buf, (size_t)len, "algo=direct_f64 n=%dx%d N=%lldx%lld batch=%lld windows_per_block=%d",
             p->n0, p->n1, (long long)p->N0, (long long)p->N1, (long long)p->batch,
             swdft::direct_f64_windows_per_block(p->n0, p->n1));
  }
  return SWDFT_OK;
}

const char* swdft2d_status_string(swdft_status_t s) {
  switch (s) {
    case SWDFT_OK: return "SWDFT_OK";
    case SWDFT_E_ARG: return "SWDFT_E_ARG";
    case SWDFT_E_NOT_POW2: return "SWDFT_E_NOT_POW2";
    case SWDFT_E_WINDOW: return "SWDFT_E_WINDOW";
    case SWDFT_E_DTYPE: return "SWDFT_E_DTYPE";
    case SWDFT_E_OVERFLOW: return "SWDFT_E_OVERFLOW";
    case SWDFT_E_NOMEM: return "SWDFT_E_NOMEM";
    case SWDFT_E_ALIGN: return "SWDFT_E_ALIGN";
    case SWDFT_E_DEVICE: return "SWDFT_E_DEVICE";
    case SWDFT_E_PLAN: return "SWDFT_E_PLAN";
    default: return "SWDFT_E_UNKNOWN";
  }
}

const char* swdft2d_last_error(void) { return g_last_error.c_str(); }

swdft_status_t swdft2d_read_probe(const void* x, int64_t bytes, float* sink, hipStream_t stream) {
  if (!x || !sink) return fail(SWDFT_E_ARG, "probe buffer or sink is null");
  if (bytes <= 0 || bytes % 8) return fail(SWDFT_E_ARG, "probe size must be a positive multiple of 8");
  if ((uintptr_t)x % 16) return fail(SWDFT_E_ALIGN, "probe buffer is not 16-byte aligned");
  if ((uintptr_t)sink % 4) return fail(SWDFT_E_ALIGN, "probe sink is not 4-byte aligned");
  hipError_t e = swdft::launch_read_probe(x, bytes, sink, stream);
  if (e != hipSuccess) return device_fail(e, "probe launch");
  return SWDFT_OK;
}

swdft_status_t swdft2d_write_probe(void* y, int64_t bytes, hipStream_t stream) {
  if (!y) return fail(SWDFT_E_ARG, "probe buffer is null");
  if (bytes <= 0 || bytes % 8) return fail(SWDFT_E_ARG, "probe size must be a positive multiple of 8");
  if ((uintptr_t)y % 8) return fail(SWDFT_E_ALIGN, "probe buffer is not 8-byte aligned");
  hipError_t e = swdft::launch_write_probe(static_cast<float2*>(y), bytes / 8, stream);
  if (e != hipSuccess) return device_fail(e, "probe launch");
  return SWDFT_OK;
}

}  // extern "C"
