// C ABI of the 3D sliding-window DFT (the k-dimensional extension of
// Sec. 4.4, k = 3): plan validation, launch shape and dispatch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_set>

#include "plan.h"

struct swdft3d_plan_s {
  int64_t N0 = 0, N1 = 0, N2 = 0, P0 = 0, P1 = 0, P2 = 0, batch = 0;
  int32_t n0 = 0, n1 = 0, n2 = 0;
  swdft_dtype_t dtype = SWDFT_R32;
  swdft_norm_t norm = SWDFT_NORM_NONE;
  swdft::Twiddles3F32 tw{};
  void* workspace = nullptr;  // adjoint partial sums, allocated at the first backward
  size_t workspace_bytes = 0;
  int workspace_device = -1;
};

namespace swdft {
namespace host {
namespace {

std::mutex g_plans3_mutex;

std::unordered_set<swdft3d_plan_s*>& live_plans3() {
  static std::unordered_set<swdft3d_plan_s*> s;
  return s;
}

bool is_live3(swdft3d_plan_t p) {
  std::lock_guard<std::mutex> lk(g_plans3_mutex);
  return p != nullptr && live_plans3().count(p) != 0;
}

// Tiles of a launch with slab length S.
int64_t tree3_tiles(const swdft3d_plan_s* p, int64_t S) {
  const int64_t nstrips = ceil_div(p->P2, tree3_columns_per_wave(p->n1, p->n2));
  return p->batch * ceil_div(p->P0, S) * p->P1 * nstrips;
}

// Resident workgroups per CU. Capped launches in dispatch order keep the
// output stream in few bands of rows: with whole columns of windows they
// raised the write rate of 128^3 / 8x8x8 from 5.4 to 6.1 TB/s and of
// 96x96x192 / 4x4x4 from 4.9 to 5.4-5.9 TB/s against uncapped launches
// (measured on gfx950); short windows along axis 0 need more waves in flight.
int32_t tree3_wpc(const swdft3d_plan_s* p) {
  const int wpc = env_int("SWDFT3D_WPC", -1);
  if (wpc >= 0) return std::min(wpc, 8);
  return p->n0 <= 4 ? 4 : 2;
}

// Window rows (axis 0) per wave when the launch is capped: slabs of 32 rows
// for n0 >= 4 (the n0-1 priming rows at a slab top compute only the levels
// its windows use, so they cost little), a whole column for n0 = 2; measured
// at 128^3 against whole columns: 8x2x8 344 -> 318 us, 8x4x8 668 -> 634 us,
// 4x4x4 179 -> 172 us, 8x8x8 1229 -> 1186 us, 16x4x4 673 -> 659 us, and
// 2x8x8 344 -> 423 us. Uncapped: enough tiles (about 4096) to fill the chip
// several times over, with slabs long enough that the priming rows stay a
// small fraction of the work. A multiple of the rows per chunk, so every
// chunk starts on a ring period.
int32_t tree3_slab(const swdft3d_plan_s* p, int wpc) {
  const int cr = tree3_rows_per_chunk(p->n0, p->n1, p->n2);
  int64_t S = env_int("SWDFT3D_SLAB", 0);
  if (S <= 0 && wpc > 0) S = p->n0 >= 4 ? 32 : p->P0;
  if (S <= 0) {
    const int64_t columns = tree3_tiles(p, p->P0);  // tiles with one slab
    S = ceil_div(p->P0 * columns, 4096);
    S = std::max<int64_t>(S, 4 * (int64_t)(p->n0 - 1));
  }
  S = std::max<int64_t>(S, cr);
  S = ceil_div(S, cr) * cr;
  S = std::min<int64_t>(S, ceil_div(p->P0, cr) * cr);
  return (int32_t)S;
}

swdft::Tree3Geom tree3_geom(const swdft3d_plan_s* p) {
  swdft::Tree3Geom g{};
  g.N0 = p->N0;
  g.N1 = p->N1;
  g.N2 = p->N2;
  g.P0 = p->P0;
  g.P1 = p->P1;
  g.P2 = p->P2;
  g.x_image_stride = p->N0 * p->N1 * p->N2;
  g.y_image_stride = p->P0 * p->P1 * p->P2 * p->n0 * p->n1 * p->n2;
  g.wpc = tree3_wpc(p);
  g.S = tree3_slab(p, g.wpc);
  g.nstrips = (int32_t)ceil_div(p->P2, tree3_columns_per_wave(p->n1, p->n2));
  g.nslabs = (int32_t)ceil_div(p->P0, g.S);
  g.batch = (int32_t)p->batch;
  g.scale = p->norm == SWDFT_NORM_ORTHO
                ? (float)(1.0 / std::sqrt((double)p->n0 * p->n1 * p->n2))
                : 1.0f;
  g.lds_cu = lds_per_cu();
  if (g.lds_cu <= 0) g.wpc = 0;
  const int64_t resident = (int64_t)g.wpc * cu_count();
  g.order = (g.wpc > 0 && resident > 0 && tree3_tiles(p, g.S) > resident) ? 1 : 0;
  return g;
}

// dx planes per wave of the 3D adjoint: a whole volume depth when the tiles
// (window rows q1 x strips) already give enough waves; otherwise slabs, each
// primed by the n0 - 1 window rows below it.
swdft::Adj3Geom adj3_geom(const swdft3d_plan_s* p) {
  swdft::Adj3Geom g{};
  g.N0 = p->N0;
  g.N1 = p->N1;
  g.N2 = p->N2;
  g.P0 = p->P0;
  g.P1 = p->P1;
  g.P2 = p->P2;
  g.y_image_stride = p->P0 * p->P1 * p->P2 * p->n0 * p->n1 * p->n2;
  g.nstrips = (int32_t)ceil_div(p->P2, tree3_columns_per_wave(p->n1, p->n2));
  const int cr = tree3_adj_rows_per_chunk(p->n0, p->n1, p->n2);
  const int64_t columns = p->batch * p->P1 * g.nstrips;
  const int64_t full = ceil_div(p->N0, cr) * cr;
  int64_t S = env_int("SWDFT3D_ADJ_SLAB", 0);
  if (S <= 0) {
    S = columns >= 1024 ? full : std::max<int64_t>(ceil_div(p->N0 * columns, 2048),
                                                    8 * (int64_t)(p->n0 - 1));
  }
  S = std::max<int64_t>(S, cr);
  S = std::min<int64_t>(ceil_div(S, cr) * cr, full);
  g.S = (int32_t)S;
  g.nslabs = (int32_t)ceil_div(p->N0, g.S);
  g.batch = (int32_t)p->batch;
  g.scale = p->norm == SWDFT_NORM_ORTHO
                ? (float)(1.0 / std::sqrt((double)p->n0 * p->n1 * p->n2))
                : 1.0f;
  g.wpc = 0;
  g.lds_cu = lds_per_cu();
  return g;
}

}  // namespace
}  // namespace host
}  // namespace swdft

using namespace swdft::host;

extern "C" {

swdft_status_t swdft3d_plan(swdft3d_plan_t* out, int64_t N0, int64_t N1, int64_t N2, int32_t n0,
                            int32_t n1, int32_t n2, swdft_dtype_t dtype, int64_t batch) {
  if (!out) return fail(SWDFT_E_ARG, "plan output pointer is null");
  *out = nullptr;
  if (N0 < 1 || N1 < 1 || N2 < 1 || n0 < 1 || n1 < 1 || n2 < 1 || batch < 1)
    return fail(SWDFT_E_ARG, "sizes must be >= 1 (N=%lld x %lld x %lld, n=%d x %d x %d, batch=%lld)",
                (long long)N0, (long long)N1, (long long)N2, n0, n1, n2, (long long)batch);
  if ((int)dtype < (int)SWDFT_R32 || (int)dtype > (int)SWDFT_C64)
    return fail(SWDFT_E_ARG, "unknown dtype %d", (int)dtype);
  if (f64_dtype(dtype)) return fail(SWDFT_E_DTYPE, "3D plans take R32 or C32 input");
  if (!is_pow2(n0) || !is_pow2(n1) || !is_pow2(n2))
    return fail(SWDFT_E_NOT_POW2, "window %d x %d x %d is not radix-2", n0, n1, n2);
  if (n0 > N0 || n1 > N1 || n2 > N2)
    return fail(SWDFT_E_WINDOW, "window %d x %d x %d larger than array %lld x %lld x %lld", n0, n1,
                n2, (long long)N0, (long long)N1, (long long)N2);
  if (!swdft::tree3_shape_supported(n0, n1, n2))
    return fail(SWDFT_E_WINDOW, "3D windows take n0 in {2,4,8,16} and n1, n2 in {2,4,8} (got %d x %d x %d)",
                n0, n1, n2);
  const int64_t P0 = N0 - n0 + 1, P1 = N1 - n1 + 1, P2 = N2 - n2 + 1;
  int64_t t = 0, elems = 0, bytes = 0, xel = 0;
  if (!mul_ok(P0, P1, &t) || !mul_ok(t, P2, &t) || !mul_ok(t, (int64_t)n0 * n1 * n2, &t) ||
      !mul_ok(t, batch, &elems) || !mul_ok(elems, 8, &bytes) || !mul_ok(N0, N1, &xel) ||
      !mul_ok(xel, N2, &xel) || !mul_ok(xel, batch, &xel) || !mul_ok(xel, 8, &xel))
    return fail(SWDFT_E_OVERFLOW, "sizes of a %lld x %lld x %lld x %lld transform overflow int64",
                (long long)batch, (long long)N0, (long long)N1, (long long)N2);
  // one workgroup per tile at the longest slabs must fit the grid
  const int64_t nstrips = (P2 + swdft::tree3_columns_per_wave(n1, n2) - 1) /
                          swdft::tree3_columns_per_wave(n1, n2);
  int64_t tiles = 0;
  if (!mul_ok(batch, P0, &tiles) || !mul_ok(tiles, P1, &tiles) || !mul_ok(tiles, nstrips, &tiles) ||
      tiles > INT32_MAX)
    return fail(SWDFT_E_OVERFLOW, "more than 2^31-1 tiles");

  auto* p = new (std::nothrow) swdft3d_plan_s();
  if (!p) return fail(SWDFT_E_NOMEM, "host allocation of the plan failed");
  p->N0 = N0;
  p->N1 = N1;
  p->N2 = N2;
  p->P0 = P0;
  p->P1 = P1;
  p->P2 = P2;
  p->n0 = n0;
  p->n1 = n1;
  p->n2 = n2;
  p->batch = batch;
  p->dtype = dtype;
  make_twiddles_f32(n0, p->tw.w0);
  make_twiddles_f32(n1, p->tw.w1);
  make_twiddles_f32(n2, p->tw.w2);
  {
    std::lock_guard<std::mutex> lk(g_plans3_mutex);
    live_plans3().insert(p);
  }
  *out = p;
  return SWDFT_OK;
}

swdft_status_t swdft3d_set_norm(swdft3d_plan_t plan, swdft_norm_t norm) {
  if (!is_live3(plan)) return fail(SWDFT_E_PLAN, "null or destroyed 3D plan");
  if (norm != SWDFT_NORM_NONE && norm != SWDFT_NORM_ORTHO)
    return fail(SWDFT_E_ARG, "unknown norm %d", (int)norm);
  plan->norm = norm;
  return SWDFT_OK;
}

int64_t swdft3d_output_elems(swdft3d_plan_t plan) {
  if (!is_live3(plan)) return -1;
  return plan->batch * plan->P0 * plan->P1 * plan->P2 * plan->n0 * plan->n1 * plan->n2;
}

swdft_status_t swdft3d_exec(swdft3d_plan_t plan, const void* x, void* y, hipStream_t stream) {
  if (!is_live3(plan)) return fail(SWDFT_E_PLAN, "null or destroyed 3D plan");
  const swdft3d_plan_s* p = plan;
  if (!x) return fail(SWDFT_E_ARG, "x is null");
  if (!y) return fail(SWDFT_E_ARG, "y is null");
  const int64_t xe = x_elem_bytes(p->dtype);
  if ((uintptr_t)x % (uintptr_t)xe)
    return fail(SWDFT_E_ALIGN, "x is not %lld-byte aligned", (long long)xe);
  if ((uintptr_t)y % 8u) return fail(SWDFT_E_ALIGN, "y is not 8-byte aligned");
  const int64_t xb = p->batch * p->N0 * p->N1 * p->N2 * xe;
  const int64_t yb = swdft3d_output_elems(plan) * 8;
  if (ranges_overlap(x, xb, y, yb)) return fail(SWDFT_E_ARG, "x and y overlap");
  const swdft::Tree3Geom g = tree3_geom(p);
  hipError_t e = swdft::launch_tree3_fwd(p->n0, p->n1, p->n2, real_dtype(p->dtype), x,
                                         static_cast<float2*>(y), g, p->tw, stream);
  if (e != hipSuccess) return device_fail(e, "3D tree launch");
  return SWDFT_OK;
}

swdft_status_t swdft3d_backward(swdft3d_plan_t plan, const void* dy, void* dx, hipStream_t stream) {
  if (!is_live3(plan)) return fail(SWDFT_E_PLAN, "null or destroyed 3D plan");
  swdft3d_plan_s* p = plan;
  if (!dy) return fail(SWDFT_E_ARG, "dy is null");
  if (!dx) return fail(SWDFT_E_ARG, "dx is null");
  const int64_t xe = x_elem_bytes(p->dtype);
  if ((uintptr_t)dy % 8u) return fail(SWDFT_E_ALIGN, "dy is not 8-byte aligned");
  if ((uintptr_t)dx % (uintptr_t)xe)
    return fail(SWDFT_E_ALIGN, "dx is not %lld-byte aligned", (long long)xe);
  const int64_t xb = p->batch * p->N0 * p->N1 * p->N2 * xe;
  const int64_t yb = swdft3d_output_elems(plan) * 8;
  if (ranges_overlap(dy, yb, dx, xb)) return fail(SWDFT_E_ARG, "dy and dx overlap");
  const swdft::Adj3Geom g = adj3_geom(p);
  int64_t ws_elems = swdft::tree3_adj_workspace_elems(p->n1, p->n2, g);
  int64_t ws_bytes = 0;
  if (!mul_ok(ws_elems, real_dtype(p->dtype) ? 4 : 8, &ws_bytes))
    return fail(SWDFT_E_OVERFLOW, "adjoint workspace size overflows int64");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (!p->workspace || p->workspace_device != dev || p->workspace_bytes < (size_t)ws_bytes) {
    if (p->workspace) {
      // the old buffer may still be read by work in flight
      e = hipDeviceSynchronize();
      if (e != hipSuccess) return device_fail(e, "hipDeviceSynchronize");
      const int cur = dev;
      if (p->workspace_device >= 0 && p->workspace_device != cur) (void)hipSetDevice(p->workspace_device);
      (void)hipFree(p->workspace);
      if (p->workspace_device != cur) (void)hipSetDevice(cur);
      p->workspace = nullptr;
      p->workspace_bytes = 0;
    }
    void* ptr = nullptr;
    e = hipMalloc(&ptr, (size_t)ws_bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(SWDFT_E_NOMEM, "3D adjoint workspace of %lld bytes: %s", (long long)ws_bytes,
                  hipGetErrorString(e));
    }
    p->workspace = ptr;
    p->workspace_bytes = (size_t)ws_bytes;
    p->workspace_device = dev;
  }
  e = swdft::launch_tree3_adj(p->n0, p->n1, p->n2, real_dtype(p->dtype),
                              static_cast<const float2*>(dy), p->workspace, dx, g, p->tw, stream);
  if (e != hipSuccess) return device_fail(e, "3D adjoint launch");
  return SWDFT_OK;
}

swdft_status_t swdft3d_describe(swdft3d_plan_t plan, char* buf, int32_t len) {
  if (!is_live3(plan)) return fail(SWDFT_E_PLAN, "null or destroyed 3D plan");
  if (!buf || len < 1) return fail(SWDFT_E_ARG, "describe buffer is null or empty");
  const swdft3d_plan_s* p = plan;
  const swdft::Tree3Geom g = tree3_geom(p);
  snprintf(buf, (size_t)len,
           "algo=tree3d n=%dx%dx%d N=%lldx%lldx%lld batch=%lld cols_per_wave=%d "
           "rows_per_chunk=%d slab=%d strips=%d slabs=%d waves=%lld groups_per_cu=%d order=%s",
           p->n0, p->n1, p->n2, (long long)p->N0, (long long)p->N1, (long long)p->N2,
           (long long)p->batch, swdft::tree3_columns_per_wave(p->n1, p->n2),
           swdft::tree3_rows_per_chunk(p->n0, p->n1, p->n2), g.S, g.nstrips, g.nslabs,
           (long long)g.batch * g.nslabs * g.P1 * g.nstrips, g.wpc, g.order ? "dispatch" : "xcd");
  return SWDFT_OK;
}

swdft_status_t swdft3d_destroy(swdft3d_plan_t plan) {
  if (plan == nullptr) return SWDFT_OK;
  {
    std::lock_guard<std::mutex> lk(g_plans3_mutex);
    auto it = live_plans3().find(plan);
    if (it == live_plans3().end()) return fail(SWDFT_E_PLAN, "3D plan already destroyed or unknown");
    live_plans3().erase(it);
  }
  swdft_status_t st = SWDFT_OK;
  if (plan->workspace) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (plan->workspace_device >= 0) (void)hipSetDevice(plan->workspace_device);
    const hipError_t e = hipFree(plan->workspace);
    if (cur >= 0) (void)hipSetDevice(cur);
    if (e != hipSuccess) st = device_fail(e, "3D workspace free");
  }
  delete plan;
  return st;
}

}  // extern "C"
