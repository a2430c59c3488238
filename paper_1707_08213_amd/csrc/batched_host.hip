// Host side of batched plans: validation, work tables, device copies and the
// graph that runs one persistent kernel per window-shape class (batched.h).
#include <algorithm>
#include <cstring>

#include "plan.h"

namespace swdft {
namespace host {

namespace {

// Output coefficients of one work item (cost used for the LPT order).
int64_t item_cost(int64_t P0, int64_t P1, int64_t rows, int64_t cols, int slab, int strip,
                  int n0, int n1) {
  const int64_t r = std::min<int64_t>(rows, P0 - (int64_t)slab * rows);
  const int64_t c = std::min<int64_t>(cols, P1 - (int64_t)strip * cols);
  return r * c * n0 * n1;
}

int device_cus(int dev) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return cus;
}

void destroy_graph(BatchState* bs) {
  if (bs->exec) (void)hipGraphExecDestroy(bs->exec);
  if (bs->graph) (void)hipGraphDestroy(bs->graph);
  bs->exec = nullptr;
  bs->graph = nullptr;
  bs->reset_node = nullptr;
  for (auto& c : bs->classes) c.node = nullptr;
  bs->gx = nullptr;
  bs->gy = nullptr;
}

const void* class_symbol(const BatchClassRun& c, bool real) {
  return c.dense ? batched_dense_symbol(c.n0, c.n1, real) : batched_tree_symbol(c.n0, c.n1, real);
}

BatchArgs class_args(const BatchState* bs, size_t i, const void* x, void* y) {
  const BatchClassRun& c = bs->classes[i];
  BatchArgs a{};
  a.x = x;
  a.y = static_cast<float2*>(y);
  a.images = bs->d_images;
  a.items = bs->d_items + c.item_begin;
  a.count = (int32_t)c.item_count;
  a.counter = bs->d_counters + i;
  a.tw = c.tw;
  return a;
}

swdft_status_t class_grid(BatchState* bs, size_t i, bool real) {
  BatchClassRun& c = bs->classes[i];
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, class_symbol(c, real), 64, 0);
  if (e != hipSuccess) return device_fail(e, "occupancy query");
  const int64_t resident = (int64_t)std::max(per_cu, 1) * device_cus(bs->device);
  c.grid = (int)std::max<int64_t>(1, std::min<int64_t>(resident, c.item_count));
  return SWDFT_OK;
}

swdft_status_t build_graph(swdft2d_plan_s* p, const void* x, void* y) {
  BatchState* bs = p->bs;
  const bool real = real_dtype(p->dtype);
  destroy_graph(bs);
  hipError_t e = hipGraphCreate(&bs->graph, 0);
  if (e != hipSuccess) return device_fail(e, "hipGraphCreate");
  int ncls = (int)bs->classes.size();
  unsigned* counters = bs->d_counters;
  void* rargs[] = {&counters, &ncls};
  hipKernelNodeParams rp{};
  rp.func = const_cast<void*>(batched_reset_symbol());
  rp.gridDim = dim3((unsigned)((ncls + 63) / 64));
  rp.blockDim = dim3(64);
  rp.sharedMemBytes = 0;
  rp.kernelParams = rargs;
  rp.extra = nullptr;
  e = hipGraphAddKernelNode(&bs->reset_node, bs->graph, nullptr, 0, &rp);
  if (e != hipSuccess) return device_fail(e, "hipGraphAddKernelNode (reset)");
  for (size_t i = 0; i < bs->classes.size(); ++i) {
    swdft_status_t st = class_grid(bs, i, real);
    if (st != SWDFT_OK) return st;
    BatchArgs a = class_args(bs, i, x, y);
    void* args[] = {&a};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(class_symbol(bs->classes[i], real));
    kp.gridDim = dim3((unsigned)bs->classes[i].grid);
    kp.blockDim = dim3(64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    e = hipGraphAddKernelNode(&bs->classes[i].node, bs->graph, &bs->reset_node, 1, &kp);
    if (e != hipSuccess) return device_fail(e, "hipGraphAddKernelNode (class)");
  }
  e = hipGraphInstantiate(&bs->exec, bs->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return device_fail(e, "hipGraphInstantiate");
  bs->gx = x;
  bs->gy = y;
  return SWDFT_OK;
}

swdft_status_t rebind_graph(swdft2d_plan_s* p, const void* x, void* y) {
  BatchState* bs = p->bs;
  const bool real = real_dtype(p->dtype);
  for (size_t i = 0; i < bs->classes.size(); ++i) {
    BatchArgs a = class_args(bs, i, x, y);
    void* args[] = {&a};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(class_symbol(bs->classes[i], real));
    kp.gridDim = dim3((unsigned)bs->classes[i].grid);
    kp.blockDim = dim3(64);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipError_t e = hipGraphExecKernelNodeSetParams(bs->exec, bs->classes[i].node, &kp);
    if (e != hipSuccess) return device_fail(e, "hipGraphExecKernelNodeSetParams");
  }
  bs->gx = x;
  bs->gy = y;
  return SWDFT_OK;
}

template <typename T>
swdft_status_t upload(T** dst, size_t* cap, const std::vector<T>& src, const char* what) {
  const size_t n = std::max<size_t>(src.size(), 1);
  if (*cap < n) {
    if (*dst) (void)hipFree(*dst);
    *dst = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), n * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(SWDFT_E_NOMEM, "%s table of %zu bytes: %s", what, n * sizeof(T),
                  hipGetErrorString(e));
    }
    *cap = n;
  }
  if (!src.empty()) {
    hipError_t e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return device_fail(e, "table upload");
  }
  return SWDFT_OK;
}

}  // namespace

int batched_default_slab(int n0, int n1, bool dense) {
  if (dense) return 64;
  const int kg = batched_tree_kg(n0, n1);
  const int cr = tree_fwd_rows_per_chunk(n0, n1, kg);
  int S = std::max(64, 4 * (n0 - 1));
  return (int)(ceil_div(S, cr) * cr);
}

void batched_build_tables(swdft2d_plan_s* p) {
  BatchState* bs = p->bs;
  const size_t count = bs->descs.size();
  bs->images.assign(count, BatchImage{});
  bs->items.clear();
  bs->classes.clear();
  std::map<std::pair<int, int>, std::vector<int64_t>> members;
  for (size_t i = 0; i < count; ++i) members[{bs->descs[i].n0, bs->descs[i].n1}].push_back((int64_t)i);

  for (auto& kv : members) {
    const int n0 = kv.first.first, n1 = kv.first.second;
    ClassCfg cfg = bs->cfg[kv.first];
    BatchClassRun run;
    run.n0 = n0;
    run.n1 = n1;
    run.dense = cfg.dense;
    make_twiddles_f32(n0, run.tw.w0);
    make_twiddles_f32(n1, run.tw.w1);
    run.item_begin = (int64_t)bs->items.size();
    const int kg = batched_tree_kg(n0, n1);
    const int cr = tree_fwd_rows_per_chunk(n0, n1, kg);
    int slab = cfg.slab > 0 ? cfg.slab : batched_default_slab(n0, n1, cfg.dense);
    std::vector<std::pair<int64_t, BatchItem>> costed;
    int64_t best = -1;
    for (int64_t i : kv.second) {
      const swdft2d_desc_t& d = bs->descs[(size_t)i];
      const int64_t P0 = d.N0 - n0 + 1, P1 = d.N1 - n1 + 1;
      BatchImage& im = bs->images[(size_t)i];
      im.x_offset = d.x_offset;
      im.y_offset = d.y_offset;
      TreeGeom& t = im.tree;
      t.N0 = d.N0;
      t.N1 = d.N1;
      t.P0 = P0;
      t.P1 = P1;
      t.x_image_stride = d.N0 * d.N1;
      t.y_image_stride = P0 * P1 * n0 * n1;
      t.kg = kg;
      int64_t S = ceil_div(std::max(slab, cr), cr) * cr;
      S = std::min<int64_t>(S, ceil_div(P0, cr) * cr);
      t.S = (int32_t)S;
      t.nstrips = (int32_t)ceil_div(P1, tree_fwd_columns_per_wave(n0, n1, kg));
      t.nslabs = (int32_t)ceil_div(P0, t.S);
      t.batch = 1;
      t.scale = norm_scale(p->norm, n0, n1);
      DenseGeom& g = im.dense;
      g.N0 = d.N0;
      g.N1 = d.N1;
      g.P0 = P0;
      g.P1 = P1;
      g.x_image_stride = d.N0 * d.N1;
      g.y_image_stride = P0 * P1 * n0 * n1;
      int64_t SD = ceil_div(std::max(slab, 16), 16) * 16;
      SD = std::min<int64_t>(SD, ceil_div(P0, 16) * 16);
      g.S = (int32_t)SD;
      g.nstrips = (int32_t)ceil_div(P1, dense_columns_per_wave(n0, n1));
      g.nslabs = (int32_t)ceil_div(P0, g.S);
      g.batch = 1;
      g.scale = t.scale;
      const int nstrips = cfg.dense ? g.nstrips : t.nstrips;
      const int nslabs = cfg.dense ? g.nslabs : t.nslabs;
      const int64_t rows = cfg.dense ? g.S : t.S;
      const int64_t cols = cfg.dense ? dense_columns_per_wave(n0, n1)
                                     : tree_fwd_columns_per_wave(n0, n1, kg);
      for (int sl = 0; sl < nslabs; ++sl)
        for (int st = 0; st < nstrips; ++st) {
          BatchItem it{(int32_t)i, st, sl, 0};
          costed.push_back({item_cost(P0, P1, rows, cols, sl, st, n0, n1), it});
        }
      if (best < 0 || P0 * P1 > (bs->descs[(size_t)best].N0 - n0 + 1) *
                                     (bs->descs[(size_t)best].N1 - n1 + 1))
        best = i;
    }
    std::stable_sort(costed.begin(), costed.end(),
                     [](const auto& a, const auto& b) { return a.first > b.first; });
    for (auto& c : costed) bs->items.push_back(c.second);
    run.item_count = (int64_t)bs->items.size() - run.item_begin;
    run.largest_image = best;
    bs->classes.push_back(run);
  }
  bs->tables_dirty = false;
  bs->device = -1;  // device copies (and the graph built on them) are stale
}

swdft_status_t batched_prepare(swdft2d_plan_s* p) {
  BatchState* bs = p->bs;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (!bs->tables_dirty && bs->device == dev) return SWDFT_OK;
  if (bs->d_images || bs->d_items || bs->d_counters) {
    // old tables and the graph may still be in use by work in flight
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return device_fail(e, "hipDeviceSynchronize");
  }
  destroy_graph(bs);
  if (bs->tables_dirty) batched_build_tables(p);
  if (bs->cap_images && bs->last_device != dev) {
    // buffers belong to another device: drop them
    if (bs->d_images) (void)hipFree(bs->d_images);
    if (bs->d_items) (void)hipFree(bs->d_items);
    if (bs->d_counters) (void)hipFree(bs->d_counters);
    bs->d_images = nullptr;
    bs->d_items = nullptr;
    bs->d_counters = nullptr;
    bs->cap_images = bs->cap_items = bs->cap_counters = 0;
  }
  swdft_status_t st = upload(&bs->d_images, &bs->cap_images, bs->images, "image");
  if (st != SWDFT_OK) return st;
  st = upload(&bs->d_items, &bs->cap_items, bs->items, "work item");
  if (st != SWDFT_OK) return st;
  std::vector<unsigned> zeros(bs->classes.size(), 0u);
  st = upload(&bs->d_counters, &bs->cap_counters, zeros, "counter");
  if (st != SWDFT_OK) return st;
  bs->device = dev;
  bs->last_device = dev;
  return SWDFT_OK;
}

swdft_status_t batched_launch_class(swdft2d_plan_s* p, size_t cls, const void* x, void* y,
                                    hipStream_t stream) {
  BatchState* bs = p->bs;
  const bool real = real_dtype(p->dtype);
  swdft_status_t st = class_grid(bs, cls, real);
  if (st != SWDFT_OK) return st;
  unsigned* counter = bs->d_counters + cls;
  int one = 1;
  void* rargs[] = {&counter, &one};
  hipError_t e = hipLaunchKernel(batched_reset_symbol(), dim3(1), dim3(64), rargs, 0, stream);
  if (e != hipSuccess) return device_fail(e, "counter reset launch");
  BatchArgs a = class_args(bs, cls, x, y);
  void* args[] = {&a};
  e = hipLaunchKernel(class_symbol(bs->classes[cls], real), dim3((unsigned)bs->classes[cls].grid),
                      dim3(64), args, 0, stream);
  if (e != hipSuccess) return device_fail(e, "class kernel launch");
  return SWDFT_OK;
}

swdft_status_t batched_exec(swdft2d_plan_s* p, const void* x, void* y, hipStream_t stream) {
  BatchState* bs = p->bs;
  if (!x) return fail(SWDFT_E_ARG, "x is null");
  if (!y) return fail(SWDFT_E_ARG, "y is null");
  if ((uintptr_t)x % (uintptr_t)x_elem_bytes(p->dtype))
    return fail(SWDFT_E_ALIGN, "x is not %lld-byte aligned", (long long)x_elem_bytes(p->dtype));
  if ((uintptr_t)y % 8) return fail(SWDFT_E_ALIGN, "y is not 8-byte aligned");
  if (ranges_overlap(x, bs->x_extent * x_elem_bytes(p->dtype), y, bs->y_extent * 8))
    return fail(SWDFT_E_ARG, "x and y overlap");
  if (!p->tuned) apply_cached_tuning(p);
  swdft_status_t st = batched_prepare(p);
  if (st != SWDFT_OK) return st;
  if (!bs->exec) {
    st = build_graph(p, x, y);
    if (st != SWDFT_OK) return st;
  } else if (bs->gx != x || bs->gy != y) {
    st = rebind_graph(p, x, y);
    if (st != SWDFT_OK) return st;
  }
  hipError_t e = hipGraphLaunch(bs->exec, stream);
  if (e != hipSuccess) return device_fail(e, "hipGraphLaunch");
  return SWDFT_OK;
}

void batched_free(BatchState* bs) {
  destroy_graph(bs);
  if (bs->d_images) (void)hipFree(bs->d_images);
  if (bs->d_items) (void)hipFree(bs->d_items);
  if (bs->d_counters) (void)hipFree(bs->d_counters);
  bs->d_images = nullptr;
  bs->d_items = nullptr;
  bs->d_counters = nullptr;
}

}  // namespace host
}  // namespace swdft

using namespace swdft::host;

extern "C" swdft_status_t swdft2d_plan_batched(swdft2d_plan_t* out, const swdft2d_desc_t* descs,
                                               int64_t count, swdft_dtype_t dtype) {
  if (!out) return fail(SWDFT_E_ARG, "plan output pointer is null");
  *out = nullptr;
  if (!descs || count < 1) return fail(SWDFT_E_ARG, "descriptor list is null or empty");
  if (count > INT32_MAX) return fail(SWDFT_E_OVERFLOW, "more than 2^31-1 images");
  if ((int)dtype < (int)SWDFT_R32 || (int)dtype > (int)SWDFT_C64)
    return fail(SWDFT_E_ARG, "unknown dtype %d", (int)dtype);
  if (f64_dtype(dtype)) return fail(SWDFT_E_DTYPE, "batched plans take R32 or C32 input");
  int64_t out_elems = 0, x_extent = 0, y_extent = 0;
  std::vector<std::pair<int64_t, int64_t>> yranges;
  for (int64_t i = 0; i < count; ++i) {
    const swdft2d_desc_t& d = descs[i];
    if (d.N0 < 1 || d.N1 < 1 || d.n0 < 1 || d.n1 < 1)
      return fail(SWDFT_E_ARG, "image %lld: sizes must be >= 1", (long long)i);
    if (!is_pow2(d.n0) || !is_pow2(d.n1))
      return fail(SWDFT_E_NOT_POW2, "image %lld: window %d x %d is not radix-2", (long long)i,
                  d.n0, d.n1);
    if (d.n0 > d.N0 || d.n1 > d.N1)
      return fail(SWDFT_E_WINDOW, "image %lld: window %d x %d larger than %lld x %lld",
                  (long long)i, d.n0, d.n1, (long long)d.N0, (long long)d.N1);
    if (!swdft::batched_shape_supported(d.n0, d.n1))
      return fail(SWDFT_E_WINDOW, "image %lld: batched plans take n0, n1 in {8, 16, 32}",
                  (long long)i);
    if (d.x_offset < 0 || d.y_offset < 0)
      return fail(SWDFT_E_ARG, "image %lld: negative offset", (long long)i);
    const int64_t P0 = d.N0 - d.n0 + 1, P1 = d.N1 - d.n1 + 1;
    int64_t o = 0, xe = 0;
    if (d.N1 > SWDFT_MAX_ROW || P0 > INT32_MAX || P1 > INT32_MAX || !mul_ok(P0, P1, &o) ||
        !mul_ok(o, (int64_t)d.n0 * d.n1, &o) || !mul_ok(d.N0, d.N1, &xe) ||
        d.x_offset > INT64_MAX / 16 - xe || d.y_offset > INT64_MAX / 16 - o ||
        out_elems > INT64_MAX / 16 - o)
      return fail(SWDFT_E_OVERFLOW, "image %lld: sizes overflow", (long long)i);
    out_elems += o;
    x_extent = std::max(x_extent, d.x_offset + xe);
    y_extent = std::max(y_extent, d.y_offset + o);
    yranges.push_back({d.y_offset, d.y_offset + o});
  }
  std::sort(yranges.begin(), yranges.end());
  for (size_t i = 1; i < yranges.size(); ++i)
    if (yranges[i].first < yranges[i - 1].second)
      return fail(SWDFT_E_ARG, "output ranges of two images overlap");

  auto* p = new (std::nothrow) swdft2d_plan_s();
  if (!p) return fail(SWDFT_E_NOMEM, "host allocation of the plan failed");
  p->kind = 1;
  p->dtype = dtype;
  p->batch = count;
  p->bs = new (std::nothrow) swdft::BatchState();
  if (!p->bs) {
    delete p;
    return fail(SWDFT_E_NOMEM, "host allocation of the plan failed");
  }
  p->bs->descs.assign(descs, descs + count);
  p->bs->out_elems = out_elems;
  p->bs->x_extent = x_extent;
  p->bs->y_extent = y_extent;
  for (int64_t i = 0; i < count; ++i) p->bs->cfg[{descs[i].n0, descs[i].n1}] = swdft::ClassCfg{};
  batched_build_tables(p);
  p->bs->tables_dirty = false;
  register_plan(p);
  *out = p;
  return SWDFT_OK;
}
