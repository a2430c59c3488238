// Host-side plan objects of libswdft2d and the helpers shared by the C ABI
// implementation files (abi.hip, batched_host.hip, tune.hip). Not part of the
// public ABI.
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "batched.h"
#include "internal.h"
#include "swdft2d.h"

namespace swdft {

// Tile choice of one window-shape class of a batched plan.
struct ClassCfg {
  bool dense = false;  // dense matrix-core variant instead of the tree
  int32_t slab = 0;    // window rows per work item (0 = default)
};

// One window-shape class present in a batched plan.
struct BatchClassRun {
  int n0 = 0, n1 = 0;
  bool dense = false;
  int64_t item_begin = 0, item_count = 0;
  int64_t largest_image = -1;  // index of the image with the most output
  TwiddlesF32 tw{};
  hipGraphNode_t node = nullptr;
  int grid = 0;
};

struct BatchState {
  std::vector<swdft2d_desc_t> descs;
  std::map<std::pair<int, int>, ClassCfg> cfg;
  std::vector<BatchImage> images;
  std::vector<BatchItem> items;
  std::vector<BatchClassRun> classes;
  int64_t out_elems = 0;  // complex outputs of all images
  int64_t x_extent = 0;   // elements of x the images span
  int64_t y_extent = 0;   // complex elements of y the images span
  bool tables_dirty = true;  // host tables must be rebuilt from descs and cfg
  int device = -1;           // device holding current copies of the tables (-1: stale)
  int last_device = -1;      // device the table buffers were allocated on
  BatchImage* d_images = nullptr;
  BatchItem* d_items = nullptr;
  unsigned* d_counters = nullptr;
  size_t cap_images = 0, cap_items = 0, cap_counters = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t reset_node = nullptr;
  const void* gx = nullptr;
  void* gy = nullptr;
};

}  // namespace swdft

struct swdft2d_plan_s {
  int kind = 0;  // 0 = images of one shape, 1 = batched uneven images
  int64_t N0 = 0, N1 = 0, P0 = 0, P1 = 0, batch = 0;
  int32_t n0 = 0, n1 = 0;
  swdft_dtype_t dtype = SWDFT_R32;
  swdft_norm_t norm = SWDFT_NORM_NONE;
  swdft_algo_t algo = SWDFT_ALGO_AUTO;
  swdft_algo_t tuned_algo = SWDFT_ALGO_AUTO;  // choice of swdft2d_tune when algo is AUTO
  bool tuned = false;                         // tuned or read from the tuning cache
  int32_t tree_slab = 0;                      // 0 = choose automatically
  int32_t tree_kg = 0;                        // 0 = choose automatically
  int32_t tree_wpc = -1;                      // resident workgroups per CU, -1 = automatic
  int32_t tree_wv = 0;                        // waves per strip (1 or 2), 0 = automatic
  int32_t dense_slab = 0;                     // 0 = choose automatically
  // Forward tree launch shape of the last exec and the inputs it was derived
  // from (device, the plan's tree_* choices, norm, SWDFT_TREE_* values): the
  // derivation costs about a microsecond of host time, as much as a small
  // image's kernel.
  bool tree_geom_valid = false;
  int32_t tree_geom_key[10] = {};
  swdft::TreeGeom tree_geom_last{};
  swdft::TwiddlesF32 tw32{};
  swdft::TwiddlesF64 tw64{};
  void* workspace = nullptr;
  size_t workspace_bytes = 0;
  int workspace_device = -1;
  swdft::BatchState* bs = nullptr;
};

namespace swdft {

// Mixed-radix (2 and 3) tree kernels (tree_mixed.hip): window shapes they
// serve (at least one side not a power of two), rows per chunk, launchers.
bool tree_mixed_supported(int n0, int n1);
int tree_mixed_rows_per_chunk(int n0, int n1);
hipError_t launch_tree_mixed_r(int n0, int n1, const void* x, float2* y, const TreeGeom& g,
                               const TwiddlesF32& tw, hipStream_t s);
hipError_t launch_tree_mixed_c(int n0, int n1, const void* x, float2* y, const TreeGeom& g,
                               const TwiddlesF32& tw, hipStream_t s);

// Lanes per column stream of the streaming kernel for windows of height n0.
int tree_stream_kg(int n0);

namespace host {

// The plan's window has a side that is not a power of two (mixed-radix tree).
bool mixed_window(const swdft2d_plan_s* p);

swdft_status_t fail(swdft_status_t st, const char* fmt, ...);
swdft_status_t device_fail(hipError_t e, const char* what);
bool is_live(swdft2d_plan_t p);
void register_plan(swdft2d_plan_s* p);
bool is_pow2(int64_t v);
bool mul_ok(int64_t a, int64_t b, int64_t* out);
bool real_dtype(swdft_dtype_t d);
bool f64_dtype(swdft_dtype_t d);
int64_t x_elem_bytes(swdft_dtype_t d);
int64_t y_elem_bytes(swdft_dtype_t d);
int64_t ceil_div(int64_t a, int64_t b);
void make_twiddles(int n, double2* w);
void make_twiddles_f32(int n, float2* w);
float norm_scale(swdft_norm_t norm, int n0, int n1);
swdft_algo_t resolve_algo(const swdft2d_plan_s* p);
TreeGeom tree_geom(const swdft2d_plan_s* p);
// tree_geom(p), derived again only when one of its inputs changed since the
// plan's last call.
const TreeGeom& tree_geom_cached(swdft2d_plan_s* p);
// Rows per chunk of the plan's tree kernel (radix-2 or mixed-radix).
int tree_chunk_rows(const swdft2d_plan_s* p, int kg, int wv);
DenseGeom dense_geom(const swdft2d_plan_s* p);
bool ranges_overlap(const void* a, int64_t abytes, const void* b, int64_t bbytes);

// batched plans (batched_host.hip)
swdft_status_t batched_exec(swdft2d_plan_s* p, const void* x, void* y, hipStream_t stream);
swdft_status_t batched_prepare(swdft2d_plan_s* p);  // tables + device copies, no graph
swdft_status_t batched_launch_class(swdft2d_plan_s* p, size_t cls, const void* x, void* y,
                                    hipStream_t stream);
void batched_build_tables(swdft2d_plan_s* p);
void batched_free(BatchState* bs);
int batched_default_slab(int n0, int n1, bool dense);

// device and environment queries (tree_config.hip)
int env_int(const char* name, int fallback);  // fallback when unset or empty
int lds_per_cu();                             // LDS bytes per CU of the current device, 0 if none
int cu_count();                               // CUs of the current device, 0 if none

// swdft2d_backward in two parts (abi.hip): every check, the launch geometry
// and the workspace bytes it needs; then the launch with a given workspace.
swdft_status_t backward_prepare(swdft2d_plan_t plan, const void* dy, void* dx, AdjGeom* g,
                                size_t* ws_bytes);
swdft_status_t backward_launch(const swdft2d_plan_s* p, const void* dy, void* ws, void* dx,
                               const AdjGeom& g, hipStream_t stream);

// tuning cache (tune.hip)
void apply_cached_tuning(swdft2d_plan_s* p);

}  // namespace host
}  // namespace swdft
