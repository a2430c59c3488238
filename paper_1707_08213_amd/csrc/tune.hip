// Autotuning of tile shapes and of the tree-versus-dense choice, with an
// accuracy gate, and a cache of the results.
//
// swdft2d_tune times candidate configurations on the caller's buffers and
// keeps the fastest. Candidates: the tree with 1 or 2 lanes per column stream,
// slab lengths from a whole column down to about 4096 tiles, resident
// workgroups per CU uncapped, 1 or 2, and one or two waves per strip; and
// (where the shape allows and the plan's
// algorithm is AUTO or DENSE) the dense matrix-core variant with its
// automatic slab and slabs of 64 to 512 window rows (fewer, longer walks are
// often faster: their store streams interleave less). The dense variant is admitted only if its output agrees with the
// tree's to a normwise relative difference of 1e-5 on the first
// min(output, 8 MiB) bytes (the tree itself is within ~2e-7 of the exact
// transform). Batched plans are tuned class by class on their own work items.
//
// Cache: when SWDFT_AUTOTUNE_CACHE names a file, results are appended to it as
// one JSON object per line, and plans consult it at their first exec:
//   {"arch":"gfx950","kind":"single","n0":16,"n1":16,"real":1,"size":20,
//    "algo":"tree","kg":1,"slab":1024,"wpc":1,"wv":1,"us":317.1}
// ("size" is floor(log2(windows per launch)); batched entries have
// "kind":"batched" and no size). The last matching line wins.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "plan.h"

namespace swdft {
namespace host {

namespace {

struct Candidate {
  bool dense = false;
  int kg = 1;
  int slab = 0;
  float us = 0.f;
  int wpc = -1;  // tree: resident workgroups per CU (0 = no cap); -1 = automatic
  int wv = 0;    // tree: waves per strip (1 or 2); 0 = automatic
};

std::string device_arch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return "unknown";
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

int size_class(int64_t windows) {
  int s = 0;
  while (windows > 1) {
    windows >>= 1;
    ++s;
  }
  return s;
}

// Median of three timed launches after one warm-up launch, in microseconds.
template <typename F>
swdft_status_t time_us(F&& launch, hipStream_t stream, float* us) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e != hipSuccess) return device_fail(e, "hipEventCreate");
  swdft_status_t st = launch();
  float t[3] = {0, 0, 0};
  for (int r = 0; r < 3 && st == SWDFT_OK; ++r) {
    e = hipEventRecord(a, stream);
    if (e == hipSuccess) st = launch();
    if (st == SWDFT_OK && e == hipSuccess) e = hipEventRecord(b, stream);
    if (st == SWDFT_OK && e == hipSuccess) e = hipEventSynchronize(b);
    if (st == SWDFT_OK && e == hipSuccess) e = hipEventElapsedTime(&t[r], a, b);
    if (e != hipSuccess && st == SWDFT_OK) st = device_fail(e, "timing");
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != SWDFT_OK) return st;
  std::sort(t, t + 3);
  *us = t[1] * 1000.f;
  return SWDFT_OK;
}

// Normwise relative difference of two complex64 host arrays.
double normwise_diff(const std::vector<float2>& a, const std::vector<float2>& ref) {
  double dmax = 0.0, rmax = 0.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double dr = (double)a[i].x - ref[i].x, di = (double)a[i].y - ref[i].y;
    dmax = std::max(dmax, std::sqrt(dr * dr + di * di));
    rmax = std::max(rmax, std::sqrt((double)ref[i].x * ref[i].x + (double)ref[i].y * ref[i].y));
  }
  return rmax > 0 ? dmax / rmax : dmax;
}

swdft_status_t copy_prefix(const void* y, size_t elems, std::vector<float2>* out) {
  out->resize(elems);
  hipError_t e = hipMemcpy(out->data(), y, elems * sizeof(float2), hipMemcpyDeviceToHost);
  return e == hipSuccess ? SWDFT_OK : device_fail(e, "hipMemcpy (accuracy gate)");
}

constexpr double kGate = 1e-5;
constexpr size_t kGateBytes = 8u << 20;
// The dense variant (error ~5e-6) must beat the tree (error ~2e-7) by this
// factor to be chosen; near-ties keep the more accurate tree.
constexpr float kDenseMargin = 0.97f;

int pick(const std::vector<Candidate>& cands, int best_tree, bool dense_ok) {
  int best = best_tree;
  for (int i = 0; i < (int)cands.size(); ++i) {
    if (!cands[i].dense || !dense_ok) continue;
    const float bar = best_tree >= 0 ? cands[best_tree].us * kDenseMargin : 3.4e38f;
    if (cands[i].us < bar && (best < 0 || cands[best].dense == false || cands[i].us < cands[best].us))
      best = i;
  }
  return best;
}

void append_cache(const std::string& line) {
  const char* path = std::getenv("SWDFT_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s\n", line.c_str());
  std::fclose(f);
}

bool json_int(const std::string& s, const char* key, long long* v) {
  const std::string k = std::string("\"") + key + "\":";
  const size_t p = s.find(k);
  if (p == std::string::npos) return false;
  return std::sscanf(s.c_str() + p + k.size(), "%lld", v) == 1;
}

bool json_str(const std::string& s, const char* key, std::string* v) {
  const std::string k = std::string("\"") + key + "\":\"";
  const size_t p = s.find(k);
  if (p == std::string::npos) return false;
  const size_t q = s.find('"', p + k.size());
  if (q == std::string::npos) return false;
  *v = s.substr(p + k.size(), q - p - k.size());
  return true;
}

swdft_status_t tune_single(swdft2d_plan_s* p, const void* x, void* y, hipStream_t stream) {
  const bool real = real_dtype(p->dtype);
  const bool allow_tree = p->algo == SWDFT_ALGO_AUTO || p->algo == SWDFT_ALGO_TREE;
  const bool allow_dense = (p->algo == SWDFT_ALGO_AUTO || p->algo == SWDFT_ALGO_DENSE_BF16X2) &&
                           dense_supported(p->n0, p->n1);
  const swdft2d_plan_s saved = *p;
  std::vector<Candidate> cands;
  if (allow_tree) {
    // slabs: the automatic choice for each cap, the whole column, and about
    // 256 to 4096 tiles; caps: none, one or two resident waves per CU
    // the mixed-radix kernels run unsplit streams on one wave per strip
    const bool mixed = mixed_window(p);
    for (int kg : {1, 2, 4, 8}) {
      if (!tree_fwd_kg_supported(p->n0, p->n1, kg) || (mixed && kg != 1)) continue;
      const int cr = tree_chunk_rows(p, kg, 1);
      const int64_t columns =
          ceil_div(p->P1, tree_fwd_columns_per_wave(p->n0, p->n1, kg)) * p->batch;
      std::vector<int64_t> slabs = {p->P0};
      for (int64_t tiles : {256, 512, 1024, 4096}) slabs.push_back(ceil_div(p->P0 * columns, tiles));
      for (int wpc : {0, 1, 2}) {
        p->tree_kg = kg;
        p->tree_wpc = wpc;
        p->tree_slab = 0;
        slabs.push_back(tree_geom(p).S);
      }
      for (int64_t s : slabs) {
        int64_t sl = ceil_div(std::max<int64_t>(s, cr), cr) * cr;
        sl = std::min<int64_t>(sl, ceil_div(p->P0, cr) * cr);
        for (int wpc : {0, 1, 2}) {
          for (int wv : {1, 2}) {
            if (!tree_fwd_wv_supported(p->n0, kg, wv) || (mixed && wv != 1)) continue;
            bool dup = false;
            for (auto& c : cands)
              dup |= (!c.dense && c.kg == kg && c.slab == sl && c.wpc == wpc && c.wv == wv);
            if (!dup) cands.push_back({false, kg, (int)sl, 0.f, wpc, wv});
          }
        }
      }
    }
  }
  if (allow_dense)
    for (int s : {0, 64, 128, 256, 512}) cands.push_back({true, 1, s, 0.f});  // 0: automatic
  auto apply = [&](const Candidate& c) {
    *p = saved;
    p->tuned = true;
    if (c.dense) {
      p->tuned_algo = SWDFT_ALGO_DENSE_BF16X2;
      p->dense_slab = c.slab;
    } else {
      p->tuned_algo = SWDFT_ALGO_TREE;
      p->tree_kg = c.kg;
      p->tree_slab = c.slab;
      p->tree_wpc = c.wpc;
      p->tree_wv = c.wv;
    }
  };
  auto run = [&]() -> swdft_status_t {
    swdft2d_plan_s* pp = p;
    return swdft2d_exec(pp, x, y, stream);
  };
  for (auto& c : cands) {
    apply(c);
    swdft_status_t st = time_us(run, stream, &c.us);
    if (st != SWDFT_OK) {
      *p = saved;
      return st;
    }
  }
  // accuracy gate for the dense candidates against the fastest tree candidate
  int best_tree = -1;
  for (int i = 0; i < (int)cands.size(); ++i)
    if (!cands[i].dense && (best_tree < 0 || cands[i].us < cands[best_tree].us)) best_tree = i;
  bool dense_ok = best_tree >= 0 ? false : true;
  if (best_tree >= 0 && allow_dense) {
    const size_t n = std::min<size_t>((size_t)swdft2d_output_elems(p), kGateBytes / sizeof(float2));
    std::vector<float2> ref, got;
    apply(cands[best_tree]);
    swdft_status_t st = run();
    if (st == SWDFT_OK) st = copy_prefix(y, n, &ref);
    Candidate dc;
    dc.dense = true;
    dc.slab = 64;
    apply(dc);
    if (st == SWDFT_OK) st = run();
    if (st == SWDFT_OK) st = copy_prefix(y, n, &got);
    if (st != SWDFT_OK) {
      *p = saved;
      return st;
    }
    dense_ok = normwise_diff(got, ref) <= kGate;
  }
  const int best = pick(cands, best_tree, dense_ok);
  if (best < 0) {
    *p = saved;
    return fail(SWDFT_E_DTYPE, "no candidate passed the accuracy gate");
  }
  apply(cands[best]);
  char line[512];
  std::snprintf(line, sizeof(line),
                "{\"arch\":\"%s\",\"kind\":\"single\",\"n0\":%d,\"n1\":%d,\"real\":%d,\"size\":%d,"
                "\"algo\":\"%s\",\"kg\":%d,\"slab\":%d,\"wpc\":%d,\"wv\":%d,\"us\":%.1f}",
                device_arch().c_str(), p->n0, p->n1, real ? 1 : 0,
                size_class(p->P0 * p->P1 * p->batch), cands[best].dense ? "dense" : "tree",
                cands[best].kg, cands[best].slab, cands[best].wpc, cands[best].wv, cands[best].us);
  append_cache(line);
  return SWDFT_OK;
}

swdft_status_t tune_batched(swdft2d_plan_s* p, const void* x, void* y, hipStream_t stream) {
  BatchState* bs = p->bs;
  const bool real = real_dtype(p->dtype);
  const bool allow_tree = p->algo == SWDFT_ALGO_AUTO || p->algo == SWDFT_ALGO_TREE;
  const bool allow_dense = p->algo == SWDFT_ALGO_AUTO || p->algo == SWDFT_ALGO_DENSE_BF16X2;
  swdft_status_t st = batched_prepare(p);
  if (st != SWDFT_OK) return st;
  const size_t ncls = bs->classes.size();
  std::vector<std::pair<int, int>> keys;
  for (const auto& c : bs->classes) keys.push_back({c.n0, c.n1});
  for (size_t ci = 0; ci < ncls; ++ci) {
    const auto key = keys[ci];
    const int n0 = key.first, n1 = key.second;
    std::vector<Candidate> cands;
    if (allow_tree) {
      const int d = batched_default_slab(n0, n1, false);
      for (int s : {d / 2, d, 2 * d}) cands.push_back({false, batched_tree_kg(n0, n1), s, 0.f});
    }
    if (allow_dense)
      for (int s : {64, 128, 256, 512}) cands.push_back({true, 1, s, 0.f});
    auto apply = [&](const Candidate& c) -> swdft_status_t {
      bs->cfg[key] = ClassCfg{c.dense, c.slab};
      bs->tables_dirty = true;
      return batched_prepare(p);
    };
    auto class_index = [&]() -> size_t {
      for (size_t i = 0; i < bs->classes.size(); ++i)
        if (bs->classes[i].n0 == n0 && bs->classes[i].n1 == n1) return i;
      return 0;
    };
    for (auto& c : cands) {
      st = apply(c);
      if (st != SWDFT_OK) return st;
      const size_t idx = class_index();
      st = time_us([&]() { return batched_launch_class(p, idx, x, y, stream); }, stream, &c.us);
      if (st != SWDFT_OK) return st;
    }
    int best_tree = -1;
    for (int i = 0; i < (int)cands.size(); ++i)
      if (!cands[i].dense && (best_tree < 0 || cands[i].us < cands[best_tree].us)) best_tree = i;
    bool dense_ok = best_tree < 0;
    if (best_tree >= 0 && allow_dense) {
      // gate on the largest image of the class
      st = apply(cands[best_tree]);
      if (st != SWDFT_OK) return st;
      size_t idx = class_index();
      const swdft2d_desc_t& d = bs->descs[(size_t)bs->classes[idx].largest_image];
      const int64_t out = (d.N0 - n0 + 1) * (d.N1 - n1 + 1) * n0 * n1;
      const size_t n = std::min<size_t>((size_t)out, kGateBytes / sizeof(float2));
      const float2* yi = static_cast<const float2*>(y) + d.y_offset;
      std::vector<float2> ref, got;
      st = batched_launch_class(p, idx, x, y, stream);
      if (st == SWDFT_OK) st = copy_prefix(yi, n, &ref);
      if (st == SWDFT_OK) st = apply(Candidate{true, 1, 64, 0.f});
      idx = class_index();
      if (st == SWDFT_OK) st = batched_launch_class(p, idx, x, y, stream);
      if (st == SWDFT_OK) st = copy_prefix(yi, n, &got);
      if (st != SWDFT_OK) return st;
      dense_ok = normwise_diff(got, ref) <= kGate;
    }
    const int best = pick(cands, best_tree, dense_ok);
    if (best < 0) return fail(SWDFT_E_DTYPE, "no candidate passed the accuracy gate");
    bs->cfg[key] = ClassCfg{cands[best].dense, cands[best].slab};
    bs->tables_dirty = true;
    char line[512];
    std::snprintf(line, sizeof(line),
                  "{\"arch\":\"%s\",\"kind\":\"batched\",\"n0\":%d,\"n1\":%d,\"real\":%d,"
                  "\"algo\":\"%s\",\"kg\":%d,\"slab\":%d,\"us\":%.1f}",
                  device_arch().c_str(), n0, n1, real ? 1 : 0,
                  cands[best].dense ? "dense" : "tree", cands[best].kg, cands[best].slab,
                  cands[best].us);
    append_cache(line);
  }
  p->tuned = true;
  return batched_prepare(p);
}

}  // namespace

void apply_cached_tuning(swdft2d_plan_s* p) {
  p->tuned = true;  // consult the cache once per plan
  if (f64_dtype(p->dtype)) return;
  const char* path = std::getenv("SWDFT_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  const std::string arch = device_arch();
  const bool real = real_dtype(p->dtype);
  char buf[1024];
  while (std::fgets(buf, sizeof(buf), f)) {
    const std::string s(buf);
    std::string a, kind, algo;
    long long n0 = 0, n1 = 0, r = 0, size = -1, kg = 1, slab = 0, wpc = -1, wv = 0;
    if (!json_str(s, "arch", &a) || a != arch || !json_str(s, "kind", &kind) ||
        !json_str(s, "algo", &algo) || !json_int(s, "n0", &n0) || !json_int(s, "n1", &n1) ||
        !json_int(s, "real", &r) || (r != 0) != real)
      continue;
    json_int(s, "kg", &kg);
    json_int(s, "slab", &slab);
    json_int(s, "wpc", &wpc);
    json_int(s, "wv", &wv);
    const bool dense = algo == "dense";
    if (p->kind == 0 && kind == "single" && n0 == p->n0 && n1 == p->n1 &&
        json_int(s, "size", &size) && size == size_class(p->P0 * p->P1 * p->batch)) {
      if (dense && !dense_supported(p->n0, p->n1)) continue;
      if (p->algo == SWDFT_ALGO_AUTO) p->tuned_algo = dense ? SWDFT_ALGO_DENSE_BF16X2 : SWDFT_ALGO_TREE;
      if (dense) {
        p->dense_slab = (int32_t)slab;
      } else if (tree_fwd_kg_supported(p->n0, p->n1, (int)kg)) {
        p->tree_kg = (int32_t)kg;
        p->tree_slab = (int32_t)slab;
        p->tree_wpc = (int32_t)wpc;
        p->tree_wv = (int32_t)wv;
      }
    } else if (p->kind == 1 && kind == "batched") {
      auto it = p->bs->cfg.find({(int)n0, (int)n1});
      if (it == p->bs->cfg.end()) continue;
      if (p->algo == SWDFT_ALGO_AUTO || (p->algo == SWDFT_ALGO_DENSE_BF16X2) == dense) {
        it->second = ClassCfg{dense, (int32_t)slab};
        p->bs->tables_dirty = true;
      }
    }
  }
  std::fclose(f);
  if (p->kind == 1 && p->bs->tables_dirty) batched_build_tables(p);
}

}  // namespace host
}  // namespace swdft

using namespace swdft::host;

extern "C" swdft_status_t swdft2d_tune(swdft2d_plan_t plan, const void* x, void* y,
                                       hipStream_t stream) {
  if (!is_live(plan)) return fail(SWDFT_E_PLAN, "null or destroyed plan");
  if (!x || !y) return fail(SWDFT_E_ARG, "x or y is null");
  if (plan->kind == 0 && f64_dtype(plan->dtype)) return SWDFT_OK;  // one algorithm: nothing to tune
  if (plan->kind == 0 && plan->algo == SWDFT_ALGO_SWFFT) return SWDFT_OK;  // one fixed shape
  const swdft_status_t st =
      plan->kind == 1 ? tune_batched(plan, x, y, stream) : tune_single(plan, x, y, stream);
  if (st != SWDFT_OK) return st;
  hipError_t e = hipStreamSynchronize(stream);
  return e == hipSuccess ? SWDFT_OK : device_fail(e, "hipStreamSynchronize");
}
