// Device tables and kernels of a batched plan: many images of uneven sizes
// and window shapes transformed by one graph launch.
//
// Images are grouped by code path (window shape and algorithm). Each group
// ("class") has its own persistent kernel: a grid of as many waves as the chip
// keeps resident pulls work items (image, window-column strip, window-row
// slab) of that class from a global counter until the class's list is
// exhausted, and runs the same tile code as the single-image kernel on each.
// Items are sorted by decreasing output bytes (longest processing time
// first). A small kernel clears the counters first; the counter reset and the
// class kernels (which depend only on the reset) form one graph.
#pragma once

#include "internal.h"

namespace swdft {

// One image of a batched plan. Read at wave-uniform addresses.
struct BatchImage {
  TreeGeom tree;      // tile geometry when the tree runs this image (batch = 1)
  DenseGeom dense;    // tile geometry when the dense variant runs it
  int64_t x_offset;   // elements of x before the image
  int64_t y_offset;   // complex64 elements of y before the image
};

// One unit of work: a tile of one image.
struct BatchItem {
  int32_t image;
  int32_t strip;
  int32_t slab;
  int32_t pad;
};

// Arguments of a class kernel (kernel parameter block).
struct BatchArgs {
  const void* x;
  float2* y;
  const BatchImage* images;
  const BatchItem* items;  // this class's items
  int32_t count;           // number of items
  int32_t pad;
  unsigned* counter;       // this class's work counter
  TwiddlesF32 tw;          // twiddles of the class's window shape
};

// Persistent class kernels exist for n0, n1 in {8, 16, 32}.
bool batched_shape_supported(int n0, int n1);
// Lanes per column stream of the tree path the batched kernels compile (fixed
// at compile time, independent of the single-plan default).
constexpr int batched_kg(int n0, int n1) { return (n0 == 32 || n0 == 8 || n1 == 8) ? 2 : 1; }
int batched_tree_kg(int n0, int n1);
// kernel symbol of a class (nullptr if none)
const void* batched_tree_symbol(int n0, int n1, bool real_input);
const void* batched_dense_symbol(int n0, int n1, bool real_input);
const void* batched_reset_symbol();

}  // namespace swdft
