// Internal declarations shared by the host plan code and the kernel files of
// libswdft2d. Nothing here is part of the public C ABI (include/swdft2d.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace swdft {

constexpr int kMaxWindow = 64;

// Twiddle vectors Omega^0 (length n0) and Omega^1 (length n1) of Sec. 4.2,
// Omega^i[m] = exp(-2 pi i m / n_i), generated in FP64 and rounded once to
// FP32. Passed to kernels by value (kernel-argument memory, read through the
// scalar cache: every twiddle a wave uses is uniform across its lanes).
struct TwiddlesF32 {
  float2 w0[kMaxWindow];
  float2 w1[kMaxWindow];
};

// Twiddle vectors of the three axes of a 3D plan.
struct Twiddles3F32 {
  float2 w0[kMaxWindow];
  float2 w1[kMaxWindow];
  float2 w2[kMaxWindow];
};

struct TwiddlesF64 {
  double2 w0[kMaxWindow];
  double2 w1[kMaxWindow];
};

// Geometry of one fused tree launch. One wave owns a strip of window columns
// (q1) and a slab of S output rows (q0) of one image.
struct TreeGeom {
  int64_t N0, N1, P0, P1;
  int64_t x_image_stride;  // elements between images of x
  int64_t y_image_stride;  // float2 between images of y
  int32_t S;               // output rows per wave
  int32_t nstrips;         // ceil(P1 / window columns per wave)
  int32_t nslabs;          // ceil(P0 / S)
  int32_t batch;
  int32_t kg;              // lanes per column stream (k0 residues), 1 or 2
  float scale;             // 1 or 1/sqrt(n0 n1)
  int32_t wpc;             // resident waves per CU: 0 = as many as fit, else capped
  int32_t lds_cu;          // LDS bytes per CU (used to impose the cap)
  int32_t order;           // tile order: 0 = a contiguous range per XCD, 1 = dispatch order
  int32_t wv;              // waves per workgroup sharing one strip, 1 or 2
};

// Geometry of one 3D forward launch. One wave owns a strip of window
// columns along axis 2 at one window row q1 of axis 1, and a slab of S window
// rows along axis 0.
struct Tree3Geom {
  int64_t N0, N1, N2, P0, P1, P2;
  int64_t x_image_stride;  // elements between volumes of x
  int64_t y_image_stride;  // float2 between volumes of y
  int32_t S;               // output rows (axis 0) per wave
  int32_t nstrips;         // ceil(P2 / window columns per wave)
  int32_t nslabs;          // ceil(P0 / S)
  int32_t batch;
  float scale;             // 1 or 1/sqrt(n0 n1 n2)
  int32_t wpc;             // resident workgroups per CU: 0 = as many as fit, else capped
  int32_t lds_cu;          // LDS bytes per CU (used to impose the cap)
  int32_t order;           // tile order: 0 = a contiguous range per XCD, 1 = dispatch order
};

// Geometry of one 3D adjoint launch. One wave owns a strip of window columns
// along axis 2 at one window row q1 of axis 1, and a slab of S planes of dx;
// it writes its partial sums for n1 x (QW + n2 - 1) x lines per plane to the
// workspace.
struct Adj3Geom {
  int64_t N0, N1, N2, P0, P1, P2;
  int64_t y_image_stride;  // float2 between volumes of dy
  int32_t S;               // dx planes per wave
  int32_t nstrips;         // ceil(P2 / windows per wave)
  int32_t nslabs;          // ceil(N0 / S)
  int32_t batch;
  float scale;
  int32_t wpc;             // resident workgroups per CU: 0 = as many as fit
  int32_t lds_cu;
};

// One call of a 2D stream: `rows` new input rows after `rows_before` rows.
struct StreamGeom {
  int64_t N1, P1;
  int64_t rows_before;     // rows the stream had received before this call
  int64_t rows;            // rows carried by this call
  int32_t nstrips;         // ceil(P1 / window columns per wave)
  float scale;             // 1 or 1/sqrt(n0 n1)
};

// Geometry of one adjoint launch. One wave owns a strip of window columns and
// a slab of S rows of dx; it writes its partial sums for the QW + n1 - 1 x
// columns its windows touch to the workspace.
struct AdjGeom {
  int64_t N0, N1, P0, P1;
  int64_t y_image_stride;  // float2 between images of dy
  int32_t S;               // dx rows per wave
  int32_t nstrips;         // ceil(P1 / window columns per wave)
  int32_t nslabs;          // ceil(N0 / S)
  int32_t batch;
  float scale;
  int32_t wpc;             // resident waves per CU: 0 = as many as fit, else capped
  int32_t lds_cu;          // LDS bytes per CU (used to impose the cap)
  int32_t kg;              // lanes per column stream (k0 residues), 1 or 2
};

// Geometry of one dense (matrix-core) launch: one wave owns 16/n1 window
// columns (one when n1 >= 16) and a slab of S window rows (S a multiple of 16).
struct DenseGeom {
  int64_t N0, N1, P0, P1;
  int64_t x_image_stride;
  int64_t y_image_stride;
  int32_t S;
  int32_t nstrips;
  int32_t nslabs;
  int32_t batch;
  float scale;
};

struct DirectGeom {
  int64_t N0, N1, P0, P1;
  int64_t x_image_stride;
  int64_t y_image_stride;
  int32_t n0, n1;
  int32_t ntiles1;  // ceil(P1 / windows per block)
  int32_t batch;
  double scale;
};

// Geometry of one per-window FFT launch (the SWFFT comparator). A workgroup
// owns a group of window columns and walks RS window rows of one image.
struct SwfftGeom {
  int64_t N0, N1, P0, P1;
  int64_t x_image_stride;  // elements between images of x
  int64_t y_image_stride;  // float2 between images of y
  int32_t RS;              // window rows per workgroup
  int32_t ngroups;         // ceil(P1 / windows per workgroup)
  int32_t nslabs;          // ceil(P0 / RS)
  int32_t batch;
  float scale;             // 1 or 1/sqrt(n0 n1)
};

// Kernel launchers (defined next to their kernels). They validate nothing:
// the plan code has checked every argument before calling them.
hipError_t launch_tree_fwd(int n0, int n1, bool real_input, const void* x, float2* y,
                           const TreeGeom& g, const TwiddlesF32& tw, hipStream_t stream);
int tree_fwd_columns_per_wave(int n0, int n1, int kg);
int tree_fwd_rows_per_chunk(int n0, int n1, int kg, int wv = 1);
// lanes per column stream used when the caller does not choose
int tree_fwd_default_kg(int n0, int n1);
bool tree_fwd_kg_supported(int n0, int n1, int kg);
bool tree_fwd_wv_supported(int n0, int kg, int wv);
int tree_fwd_resident_waves(int wpc, int ncu);

// streaming 2D tree (tree_stream.hip)
int tree_stream_state_slots(int n0);  // ring values per lane (m0 n0 / 2, at least 1)
hipError_t launch_tree_stream(int n0, int n1, bool real_input, const void* x, float2* y,
                              float2* state, const StreamGeom& g, const TwiddlesF32& tw,
                              hipStream_t stream);
hipError_t launch_fill_zero(float2* p, int64_t n, hipStream_t stream);

// 3D forward tree (tree3d_fwd.hip)
bool tree3_shape_supported(int n0, int n1, int n2);
int tree3_columns_per_wave(int n1, int n2);
int tree3_rows_per_chunk(int n0, int n1, int n2);
hipError_t launch_tree3_fwd(int n0, int n1, int n2, bool real_input, const void* x, float2* y,
                            const Tree3Geom& g, const Twiddles3F32& tw, hipStream_t stream);

// 3D adjoint (tree3d_adj.hip)
int tree3_adj_rows_per_chunk(int n0, int n1, int n2);
int64_t tree3_adj_workspace_elems(int n1, int n2, const Adj3Geom& g);
hipError_t launch_tree3_adj(int n0, int n1, int n2, bool real_input, const float2* dy, void* ws,
                            void* dx, const Adj3Geom& g, const Twiddles3F32& tw,
                            hipStream_t stream);

hipError_t launch_tree_adj(int n0, int n1, bool real_input, const float2* dy, void* ws, void* dx,
                           const AdjGeom& g, const TwiddlesF32& tw, hipStream_t stream);
int tree_adj_rows_per_chunk(int n0, int n1, int kg);
int tree_adj_columns_per_wave(int n0, int n1, int kg);
int tree_adj_default_kg(int n0, int n1);
bool tree_adj_kg_supported(int n0, int n1, int kg);
// workspace elements (float for real input, float2 for complex) of one adjoint launch
int64_t tree_adj_workspace_elems(int n0, int n1, const AdjGeom& g);

hipError_t launch_dense_fwd(int n0, int n1, bool real_input, const void* x, float2* y,
                            const DenseGeom& g, const TwiddlesF32& tw, hipStream_t stream);
bool dense_supported(int n0, int n1);
int dense_columns_per_wave(int n0, int n1);

hipError_t launch_direct_f64(int n0, int n1, bool real_input, const void* x, double2* y,
                             const DirectGeom& g, const TwiddlesF64& tw, hipStream_t stream);
int direct_f64_windows_per_block(int n0, int n1);

hipError_t launch_swfft(int n0, int n1, bool real_input, const void* x, float2* y,
                        const SwfftGeom& g, const TwiddlesF32& tw, hipStream_t stream);
int swfft_windows_per_group(int n0, int n1);

hipError_t launch_write_probe(float2* y, int64_t n_float2, hipStream_t stream);
hipError_t launch_read_probe(const void* x, int64_t bytes, float* sink, hipStream_t stream);

}  // namespace swdft
