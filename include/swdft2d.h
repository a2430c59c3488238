/*
 * swdft2d.h - C ABI of the MI355X (gfx950) 2D Tree Sliding-Window DFT library.
 *
 * Problem (Sec. 4.1, Eq. (2)): for an N0 x N1 array x and radix-2 windows
 * n0 = 2^m0, n1 = 2^m1 (n_i <= N_i, non-square allowed), or mixed-radix
 * windows whose sides are 2^a 3^b (Sec. 5; see swdft2d_plan), compute for
 * every window position the 2D DFT of that n0 x n1 window:
 *
 *   y[b][q0][q1][k0][k1] = s * sum_{j0<n0} sum_{j1<n1} x[b][q0+j0][q1+j1]
 *                          * exp(-2 pi i (j0 k0 / n0 + j1 k1 / n1))
 *
 * with q_i = p_i - n_i + 1 in [0, P_i), P_i = N_i - n_i + 1 (the paper indexes
 * windows by their bottom-right corner p_i; the output is stored by the
 * top-left corner q_i), k_i in [0, n_i). s = 1 by default (the tree's natural,
 * unnormalised output, which equals a per-window FFT, Sec. 4.6) or
 * s = 1/sqrt(n0 n1) (the scale printed in Eq. (2)), see swdft2d_set_norm.
 * The output holds P0*P1*n0*n1 coefficients per image (Sec. 4.1, Sec. 4.3).
 *
 * Algorithms (swdft2d_set_algo):
 *   TREE   - the 2D Tree SWDFT: log2(n1) row levels (Eq. (5)) then log2(n0)
 *            column levels (Eq. (6)) swept over the whole grid so every
 *            sub-DFT shared by overlapping windows is computed once per tile.
 *            FP32 arithmetic, twiddles generated in FP64 and rounded once.
 *            Sides with a factor 3 run ternary levels (3-point butterflies)
 *            after the binary ones.
 *   DENSE_BF16X2 - each window as F_n0 X F_n1^T on the matrix cores, BF16
 *            hi/lo split products accumulated in FP32 (n0, n1 in {8,16,32};
 *            normwise relative error about 5e-6 instead of the tree's 2e-7).
 *   DIRECT_F64 - Eq. (2) evaluated literally per coefficient in FP64
 *            (the comparator; the only algorithm for R64/C64 input).
 *   SWFFT  - the 2D SWFFT comparator of Table 1 and Fig. 4: a radix-2
 *            row-column FFT of every window from scratch, nothing shared
 *            between windows, (n0 n1 / 2) log2(n0 n1) butterflies per window.
 *            FP32, the same twiddles and butterflies as the tree, so it
 *            computes the same intermediate values (Sec. 4.6).
 *   AUTO   - TREE for R32/C32, DIRECT_F64 for R64/C64.
 *
 * Memory layout (all row-major, contiguous, device memory owned by the caller):
 *   x  : [batch][N0][N1]  float (R32), float2 interleaved (C32),
 *                         double (R64), double2 (C64)
 *   y  : [batch][P0][P1][n0][n1] complex, k1 fastest:
 *                         float2 for R32/C32, double2 for R64/C64
 *   dx : layout and type of x; dy : layout and type of y.
 * For real x the full n0 x n1 spectrum is written (no Hermitian packing).
 *
 * Ownership: the caller owns x, y, dx, dy. A plan owns only host state and,
 * once backward has run, a device workspace it frees in swdft2d_destroy.
 * Plans never allocate at creation, so plan-time validation needs no GPU.
 *
 * Streams: exec and backward only enqueue work on the given stream (0 = the
 * null stream) and never synchronise. The caller must not destroy a plan, nor
 * free its buffers, while work enqueued with it is in flight. Calls with one
 * plan from several host threads must be serialised by the caller. All
 * swdft2d_backward calls of one plan share its one workspace: calls on
 * different streams must be ordered by the caller (events), or each stream
 * should use a plan of its own.
 *
 * Errors: every entry point returns a status and never aborts. All argument
 * checks happen on the host before anything is enqueued; on an error nothing
 * is enqueued and outputs are untouched. swdft2d_last_error() gives a
 * thread-local detail string for the last failing call on this thread.
 *
 * Environment variables read by the library. None changes what is computed;
 * the SWDFT_*_SLAB / TREE_* ones change only the launch shape (and so, for
 * the tree, nothing but the order of independent work), and are read each
 * time a plan derives its launch shape (at every exec). A value the shape
 * has no kernel for falls back to the default; a plan's own tuned choice
 * (swdft2d_tune or the cache) takes precedence over them.
 *   SWDFT_AUTOTUNE_CACHE  path of the JSON-lines tuning cache (swdft2d_tune)
 *   SWDFT_TREE_KG         lanes per column stream of the forward tree (1 or 2;
 *                         n0 = 64 plans have one split per n1)
 *   SWDFT_TREE_WPC        resident workgroups per CU of the forward tree
 *                         (0 = no cap, 1..8)
 *   SWDFT_TREE_WV         waves per strip of the forward tree (1 or 2)
 *   SWDFT_TREE_SLAB       window rows per workgroup of the forward tree
 *   SWDFT_ADJ_SLAB        dx rows per workgroup of swdft2d_backward
 *   SWDFT_ADJ_KG          lanes per column stream of swdft2d_backward (1 or 2;
 *                         2 is built for n0 >= 8 with n1 <= 32)
 *   SWDFT_ADJ_WPC         resident workgroups per CU of swdft2d_backward
 *                         (0 = no cap)
 *   SWDFT_DENSE_SLAB      window rows per workgroup of DENSE_BF16X2
 *   SWDFT3D_WPC           resident workgroups per CU of swdft3d_exec
 *   SWDFT3D_SLAB          window rows (axis 0) per workgroup of swdft3d_exec
 *   SWDFT3D_ADJ_SLAB      dx planes per workgroup of swdft3d_backward
 */
#ifndef SWDFT2D_H
#define SWDFT2D_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SWDFT_R32 = 0, /* real float input, complex64 output */
    SWDFT_C32 = 1, /* complex64 input, complex64 output */
    SWDFT_R64 = 2, /* real double input, complex128 output (DIRECT_F64 only) */
    SWDFT_C64 = 3  /* complex128 input, complex128 output (DIRECT_F64 only) */
} swdft_dtype_t;

typedef enum {
    SWDFT_NORM_NONE = 0,  /* s = 1: the tree's natural output (default) */
    SWDFT_NORM_ORTHO = 1  /* s = 1/sqrt(n0 n1), as printed in Eq. (2) */
} swdft_norm_t;

typedef enum {
    SWDFT_ALGO_AUTO = 0,
    SWDFT_ALGO_TREE = 1,
    SWDFT_ALGO_DENSE_BF16X2 = 2,
    SWDFT_ALGO_DIRECT_F64 = 3,
    SWDFT_ALGO_SWFFT = 4
} swdft_algo_t;

typedef int swdft_status_t;
#define SWDFT_OK 0
#define SWDFT_E_ARG 1         /* null pointer, size <= 0, unknown enum value */
#define SWDFT_E_NOT_POW2 2    /* window shape is neither radix-2 (Sec. 4.1) nor one of
                                 the mixed-radix shapes of swdft2d_plan */
#define SWDFT_E_WINDOW 3      /* n_i > N_i, or n_i above SWDFT_MAX_WINDOW */
#define SWDFT_E_DTYPE 4       /* dtype / algorithm combination not supported */
#define SWDFT_E_OVERFLOW 5    /* element or byte count does not fit in int64 */
#define SWDFT_E_NOMEM 6       /* workspace allocation failed */
#define SWDFT_E_ALIGN 7       /* a buffer is not aligned to its element size */
#define SWDFT_E_DEVICE 8      /* a HIP call failed; detail in swdft2d_last_error() */
#define SWDFT_E_PLAN 9        /* null or destroyed plan, or wrong plan kind */

#define SWDFT_MAX_WINDOW 64   /* largest n0 or n1 a plan accepts */
#define SWDFT_MAX_WINDOW_ADJ 32 /* largest n0 or n1 of swdft2d_backward and of
                                   2D streams */
#define SWDFT_MAX_ROW 2097152 /* largest N1 a plan accepts: 128 input rows of it
                                 (the most one tile stages) stay within 2 GiB,
                                 so kernels address them with 32-bit offsets */

typedef struct swdft2d_plan_s* swdft2d_plan_t;

/* Create a plan for `batch` images of N0 x N1 with n0 x n1 windows.
 * Checks, in this order: out != NULL (E_ARG); N0, N1, n0, n1, batch >= 1 and
 * dtype known (E_ARG); n0, n1 powers of two, or both from {3, 4, 6, 8, 9, 12,
 * 16, 24} with at least one of them in {3, 6, 9, 12, 24} (E_NOT_POW2: the
 * mixed-radix tree; such plans run TREE or DIRECT_F64 forward only, and
 * swdft2d_backward, SWFFT and DENSE_BF16X2 return E_WINDOW); n_i <= N_i and
 * n_i <= SWDFT_MAX_WINDOW (E_WINDOW); batch*P0*P1*n0*n1 and its byte count fit
 * in int64, and N1 <= SWDFT_MAX_ROW (E_OVERFLOW). Builds the twiddle vectors
 * Omega^0, Omega^1 of Sec. 4.2 in FP64 (exact at quarter turns, Omega[m + n/2] = -Omega[m]) and
 * rounds them once to FP32. Touches no GPU. On error *out is set to NULL. */
swdft_status_t swdft2d_plan(swdft2d_plan_t* out, int64_t N0, int64_t N1, int32_t n0, int32_t n1,
                            swdft_dtype_t dtype, int64_t batch);

/* Select the output scale. Allowed at any time; affects later calls. */
swdft_status_t swdft2d_set_norm(swdft2d_plan_t plan, swdft_norm_t norm);

/* Select the algorithm. E_DTYPE if it cannot serve the plan's dtype (TREE,
 * DENSE_BF16X2 and SWFFT serve R32/C32; DIRECT_F64 serves R64/C64, whose callers widen
 * FP32 data to FP64 exactly beforehand); E_WINDOW if DENSE_BF16X2 is asked for
 * a window outside {8,16,32} x {8,16,32}, or SWFFT for a window that is not
 * radix-2. */
swdft_status_t swdft2d_set_algo(swdft2d_plan_t plan, swdft_algo_t algo);

/* Forward transform: x (layout above) -> y. Enqueued on `stream`.
 * E_ARG for null x or y, E_ALIGN if x or y is not aligned to its element
 * size (4/8/8/16 bytes for x by dtype; 8 or 16 bytes for y), E_ARG if the
 * byte ranges of x and y overlap. */
swdft_status_t swdft2d_exec(swdft2d_plan_t plan, const void* x, void* y, hipStream_t stream);

/* Adjoint of the forward map (the conjugate transpose M^H of the linear map
 * x -> y of Eq. (2) with the plan's scale): dy (layout of y) -> dx (layout of
 * x). For real dtypes dx = Re(M^H dy), the gradient of a real loss L with
 * respect to x when dy = dL/dRe(y) + i dL/dIm(y). Computed with the levels of
 * Eq. (5)-(6) transposed and run in reverse (gather form: deterministic, no
 * atomics). Supported for R32/C32 plans with TREE (or AUTO); E_DTYPE
 * otherwise. E_WINDOW for n_i above SWDFT_MAX_WINDOW_ADJ or a window that is
 * not radix-2 (checked first, after the plan itself). Errors as for exec. Allocates the plan's workspace (partial sums
 * of (64/n1 + n1 - 1) x-columns per strip of 64/n1 window columns, about
 * (1 + n1^2/64) times the size of dx) on first use, or when called on another
 * device, with hipMalloc (E_NOMEM on failure); later calls reuse it. */
swdft_status_t swdft2d_backward(swdft2d_plan_t plan, const void* dy, void* dx, hipStream_t stream);

/* Free the plan and its workspace. Null is accepted (no-op). The caller must
 * make sure no work enqueued with the plan is still running. */
swdft_status_t swdft2d_destroy(swdft2d_plan_t plan);

/* batch*P0*P1*n0*n1 (sum over images for a batched plan), or -1 for a null
 * plan. */
int64_t swdft2d_output_elems(swdft2d_plan_t plan);

/* Byte size of y (output_elems times 8 or 16), or -1 for a null plan. */
int64_t swdft2d_output_bytes(swdft2d_plan_t plan);

/* Write a one-line description of the plan's resolved kernel and tiling into
 * buf (NUL-terminated, truncated to len). Returns the status. */
swdft_status_t swdft2d_describe(swdft2d_plan_t plan, char* buf, int32_t len);

/* Human-readable name of a status code (static storage). */
const char* swdft2d_status_string(swdft_status_t status);

/* Detail of the last failing call on the calling thread ("" if none). */
const char* swdft2d_last_error(void);

/* One image of a batched plan. Offsets count elements of the caller's packed
 * x (of the plan's dtype) and complex elements of the packed y; image i's
 * input is x[x_offset .. x_offset + N0*N1) row-major and its output is
 * y[y_offset .. y_offset + P0*P1*n0*n1) in the layout of a single-image plan.
 * Output ranges of different images must not overlap. */
typedef struct {
    int64_t N0, N1;     /* image size */
    int32_t n0, n1;     /* window size, each in {8, 16, 32} */
    int64_t x_offset;   /* elements of x before this image */
    int64_t y_offset;   /* complex elements of y before this image */
} swdft2d_desc_t;

/* Plan for `count` images of uneven sizes and window shapes, transformed by
 * one exec. dtype must be R32 or C32 (E_DTYPE otherwise). Checks each
 * descriptor as swdft2d_plan does (E_ARG, E_NOT_POW2, E_WINDOW), rejects
 * window sizes outside {8,16,32} (E_WINDOW), negative offsets and overlapping
 * output ranges (E_ARG), and sizes that overflow int64 or N1 above
 * SWDFT_MAX_ROW (E_OVERFLOW). Images
 * are grouped by window shape; each group runs its own persistent kernel (a
 * grid of the waves the chip keeps resident pulling tiles from a work list
 * sorted by decreasing output bytes). At the first exec the plan uploads its
 * work tables (hipMalloc, owned by the plan) and builds a graph of a
 * counter-reset kernel followed by the group kernels; each exec is one
 * hipGraphLaunch on the stream. Exec with other x/y pointers rebinds the
 * graph's arguments. backward is not available (E_PLAN). Touches no GPU. */
swdft_status_t swdft2d_plan_batched(swdft2d_plan_t* out, const swdft2d_desc_t* descs, int64_t count,
                                    swdft_dtype_t dtype);

/* Time candidate configurations on the caller's x and y and keep the fastest:
 * tree tile shapes (lanes per column stream, slab length, resident
 * workgroups per CU, waves per strip) and, when the
 * plan's algorithm is AUTO (or DENSE_BF16X2) and the window shape allows, the
 * dense matrix-core variant, which is admitted only if its output agrees with
 * the tree's to a normwise relative difference of 1e-5. Batched plans are
 * tuned per window-shape group. y is overwritten. Blocks until the stream is
 * idle. Results are appended to the file named by SWDFT_AUTOTUNE_CACHE (one
 * JSON object per line) when it is set; plans read that file at their first
 * exec. R64/C64 plans have nothing to tune (returns SWDFT_OK). */
swdft_status_t swdft2d_tune(swdft2d_plan_t plan, const void* x, void* y, hipStream_t stream);

/* For callers that cannot allocate device memory (work recorded under
 * stream capture, serving loops that forbid allocation): swdft2d_backward
 * with its workspace in a fixed array of the library, one per device
 * (SWDFT_NOALLOC_SCRATCH_BYTES bytes, held from the first call on a device
 * until the process ends), instead of a plan-owned allocation. Arguments,
 * layouts, checks and result are those of swdft2d_backward (the same
 * kernels and launch shape: dx is bitwise equal). It calls no allocation
 * routine; the first call on a device looks up the array's device address.
 * Checks: those of swdft2d_backward, then E_NOMEM when the adjoint's
 * workspace exceeds SWDFT_NOALLOC_SCRATCH_BYTES: batch * ceil(P1 / W) * N0 *
 * (W + n1 - 1) elements of 4 bytes (R32) or 8 bytes (C32), W = 64 / (n1 kg)
 * window columns per strip, kg = 2 for n0 = 32 and 1 otherwise (about 19 MB
 * for 1024 x 1024 with 16 x 16 windows). Nothing is enqueued on an error.
 * All calls on one device share that device's array: calls that overlap in
 * time on one device (other streams, other threads, other plans) race and
 * give wrong results; order them. The array keeps the last call's contents
 * (every call overwrites all of it that it reads). */
#define SWDFT_NOALLOC_SCRATCH_BYTES (32u * 1024u * 1024u)
swdft_status_t swdft2d_backward_noalloc(swdft2d_plan_t plan, const void* dy, void* dx,
                                        hipStream_t stream);

/* Copy the plan's FP32 twiddle vector of one axis (Sec. 4.2: Omega^0 for
 * axis 0, length n0; Omega^1 for axis 1, length n1) into out as interleaved
 * (re, im) floats, out[2m] + i out[2m+1] = Omega[m] = exp(-2 pi i m / n)
 * generated in FP64 and rounded once to nearest-even: exactly 1 at m = 0, -i
 * at m = n/4, and Omega[m + n/2] = -Omega[m] for even n. These are the values
 * every FP32 kernel of the plan multiplies by. Read-only; touches no GPU.
 * Checks: live single-image plan (E_PLAN); axis 0 or 1, out != NULL and
 * len >= 2 n (E_ARG). */
swdft_status_t swdft2d_twiddles(swdft2d_plan_t plan, int32_t axis, float* out, int32_t len);

/* Measurement aid (not part of the transform): fill `bytes` bytes at y
 * (8-byte aligned, bytes a multiple of 8) with a constant, with the access
 * pattern of a device memset (16-byte stores, 256 workgroups sweeping the
 * buffer front to back). Timing it gives the empirical HBM write ceiling at a
 * given byte count. */
swdft_status_t swdft2d_write_probe(void* y, int64_t bytes, hipStream_t stream);

/* Measurement aid (not part of the transform): read `bytes` bytes at x
 * (16-byte aligned, bytes a multiple of 8) with non-temporal 16-byte loads
 * (16384 workgroups of 256 lanes sweeping the buffer front to back). Nothing
 * is written in practice: *sink (device memory, 4-byte aligned) is stored to
 * only if the sum of the values read is one particular NaN bit pattern.
 * Timing it gives the empirical HBM read ceiling at a given byte count, the
 * bound of swdft2d_backward's input stream. Checks: x, sink non-null and
 * bytes > 0, a multiple of 8 (E_ARG); alignment (E_ALIGN). */
swdft_status_t swdft2d_read_probe(const void* x, int64_t bytes, float* sink, hipStream_t stream);

/* ---- Streaming 2D sliding-window DFT: the order of Sec. 4.3 in which the
 * loops over trees are innermost, for rows that arrive one after another
 * (a real-time task). The column-level state of the trees (m0 n0 / 2 complex
 * values per (window column, k1) stream, m0 = log2 n0) stays resident on the
 * device between
 * calls; each call carries any number of new rows and emits every window row
 * they complete: with R rows after B rows, the window rows q0 in
 * [max(0, B - n0 + 1), max(0, B + R - n0 + 1)). The emitted values equal
 * those of swdft2d_exec on the concatenated rows. */
typedef struct swdft2d_stream_s* swdft2d_stream_t;

/* Checks: out != NULL, N1, n0, n1 >= 1 and dtype known (E_ARG); dtype R32 or
 * C32 (E_DTYPE); n0, n1 powers of two (E_NOT_POW2); n1 <= N1 and
 * n_i <= SWDFT_MAX_WINDOW_ADJ (E_WINDOW); N1 <= SWDFT_MAX_ROW (E_OVERFLOW).
 * Touches no GPU. The device state, 8 * max(m0 n0 / 2, 1) * 64 bytes per strip
 * of 64/n1 window columns for n0 < 4 (about 4 m0 n0 n1 (N1 - n1 + 1) bytes;
 * from n0 = 4 on each stream is split over two lanes, which keep 1.2 to 1.5
 * times that in all), is allocated with hipMalloc at the first push, on the
 * current device, and cleared there with a kernel. */
swdft_status_t swdft2d_stream_create(swdft2d_stream_t* out, int64_t N1, int32_t n0, int32_t n1,
                                     swdft_dtype_t dtype);

/* Select the output scale; affects later pushes. */
swdft_status_t swdft2d_stream_set_norm(swdft2d_stream_t s, swdft_norm_t norm);

/* Rows received so far (-1 for a null or destroyed stream). */
int64_t swdft2d_stream_rows(swdft2d_stream_t s);

/* Window rows that a push of `rows` rows would emit now (-1 on bad input). */
int64_t swdft2d_stream_completes(swdft2d_stream_t s, int64_t rows);

/* Append `rows` rows x[rows][N1] (device memory, float or float2) and enqueue
 * on `stream` the kernel that writes the window rows they complete to
 * y[count][P1][n0][n1] (complex64, count = swdft2d_stream_completes(s, rows)
 * before the call; y may be NULL when count is 0). Pushes of one stream must
 * execute in order (one HIP stream, or synchronised) and on the device that
 * holds the state (E_ARG otherwise). rows = 0 is a no-op. */
swdft_status_t swdft2d_stream_push(swdft2d_stream_t s, const void* x, int64_t rows, void* y,
                                   hipStream_t stream);

/* Start over with no rows: clears the state with a kernel on `stream`. */
swdft_status_t swdft2d_stream_reset(swdft2d_stream_t s, hipStream_t stream);

/* Free the stream and its device state (E_PLAN if already destroyed; NULL is
 * accepted). The caller must not destroy it while its work is in flight. */
swdft_status_t swdft2d_stream_destroy(swdft2d_stream_t s);

/* ---- 3D sliding-window DFT: the k-dimensional extension of Sec. 4.4 with
 * k = 3. Its trees run the levels of axis 2, then axis 1, then axis 0 (the
 * three instances of Eq. (7) printed there) and end in the 3D DFT of every
 * window:
 *   y[b][q0][q1][q2][k0][k1][k2] = s * sum_{j<n} x[b][q0+j0][q1+j1][q2+j2]
 *                                  * W0^(j0 k0) W1^(j1 k1) W2^(j2 k2)
 * with W_n = exp(-2 pi i / n) and s = 1 (NONE) or 1/sqrt(n0 n1 n2) (ORTHO).
 * x is [batch][N0][N1][N2] row-major (float for R32, float2 for C32); y is
 * [batch][P0][P1][P2][n0][n1][n2] complex64, P_i = N_i - n_i + 1, k2 fastest.
 * The caller owns x and y; y must not overlap x. */
typedef struct swdft3d_plan_s* swdft3d_plan_t;

/* Checks, in this order: out != NULL (E_ARG); sizes >= 1 and dtype known
 * (E_ARG); dtype R32 or C32 (E_DTYPE); n_i powers of two (E_NOT_POW2);
 * n_i <= N_i, n0 in {2, 4, 8, 16} and n1, n2 in {2, 4, 8} (E_WINDOW); element,
 * byte and tile counts fit (E_OVERFLOW). Builds the twiddle vectors of the
 * three axes in FP64 and rounds them once to FP32. Touches no GPU. On error
 * *out is set to NULL. */
swdft_status_t swdft3d_plan(swdft3d_plan_t* out, int64_t N0, int64_t N1, int64_t N2, int32_t n0,
                            int32_t n1, int32_t n2, swdft_dtype_t dtype, int64_t batch);

/* Select the output scale; affects later execs. */
swdft_status_t swdft3d_set_norm(swdft3d_plan_t plan, swdft_norm_t norm);

/* Enqueue the transform on `stream` (no synchronisation). x must be aligned
 * to its element size and y to 8 bytes (E_ALIGN); null pointers and
 * overlapping x/y give E_ARG; a failed launch gives E_DEVICE. */
swdft_status_t swdft3d_exec(swdft3d_plan_t plan, const void* x, void* y, hipStream_t stream);

/* batch*P0*P1*P2*n0*n1*n2, or -1 for a null or destroyed plan. */
int64_t swdft3d_output_elems(swdft3d_plan_t plan);

/* Launch shape as text (algorithm, tile, slab, counts). */
swdft_status_t swdft3d_describe(swdft3d_plan_t plan, char* buf, int32_t len);

/* Adjoint of the 3D map x -> y (its conjugate transpose, the 3D analogue of
 * swdft2d_backward): dx = M^H dy, Re(M^H dy) for an R32 plan. dy has y's
 * layout [batch][P0][P1][P2][n0][n1][n2] (complex64), dx has x's layout and
 * type. The transposed tree levels run in reverse order (axis 0 streamed up
 * each slab, then axes 1 and 2 per window position), and partial sums per
 * (window row q1, strip) tile go through a plan-owned workspace (about
 * n1 (W + n2 - 1) / W times dx, W = 64 / (n1 n2)) allocated at the first
 * call and freed by swdft3d_destroy; a second kernel adds them in a fixed
 * order (deterministic). Checks: live plan (E_PLAN); dy, dx non-null (E_ARG),
 * dy 8-byte and dx element aligned (E_ALIGN), not overlapping (E_ARG);
 * E_NOMEM when the workspace cannot be allocated. Calls with one plan must
 * be ordered (they share its workspace). */
swdft_status_t swdft3d_backward(swdft3d_plan_t plan, const void* dy, void* dx, hipStream_t stream);

/* Free the plan (E_PLAN if already destroyed). NULL is accepted. The caller
 * must not destroy a plan while work it enqueued is in flight. */
swdft_status_t swdft3d_destroy(swdft3d_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* SWDFT2D_H */
