/*
 * FP64 oracle for the 2D sliding-window DFT (2D SWDFT), and for its 3D
 * extension (Sec. 4.4).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the bench's
 * CPU-baseline leg may load this code; the product path never does. It shares
 * no code, header, table or helper with the GPU library.
 *
 * What it computes is the plain definition, Eq. (2) of Sec. 4.1, evaluated
 * window by window with no fast algorithm:
 *
 *   a[q0][q1][k0][k1] = s * sum_{j0<n0} sum_{j1<n1} x[q0+j0][q1+j1]
 *                              * W0[(j0*k0) mod n0] * W1[(j1*k1) mod n1]
 *
 * with W_n[m] = exp(-2*pi*i*m/n), q_i = p_i - n_i + 1 the top-left corner of
 * the window whose bottom-right corner is p_i (Sec. 4.1), and
 * s = 1 (unnormalised, what the tree of Eq. (5)-(6) produces) or
 * s = 1/sqrt(n0*n1) (the scale printed in Eq. (2)).
 *
 * Readings taken where the paper is loose (each is listed in the design notes):
 *  - the twiddle is the forward-DFT root exp(-2*pi*i/n), k < n (Sec. 3.1 prints
 *    a garbled root with N in place of n);
 *  - the default is unnormalised; the 1/sqrt(n0 n1) of Eq. (2) is an option.
 *
 * The adjoint is the explicit conjugate transpose of that same linear map:
 *
 *   dx[r][c] = s * sum_{windows (q0,q1) covering (r,c)} sum_{k0,k1}
 *              dy[q0][q1][k0][k1] * conj(W0[((r-q0)*k0) mod n0] * W1[((c-q1)*k1) mod n1])
 *
 * Sums run sequentially in FP64 in the order written. Windows (or pixels) are
 * independent and are spread over threads with OpenMP; that changes no
 * arithmetic. The transform itself does not need n to be a power of two, so
 * the oracle accepts any 1 <= n_i <= N_i.
 *
 * Compile-time switch ORACLE_MUTATION (tests only): builds a deliberately
 * wrong variant so the tests can show that their pins catch such mistakes.
 * The default build (no macro) contains none of it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifndef ORACLE_MUTATION
#define ORACLE_MUTATION 0
#endif

#define ORACLE_OK 0
#define ORACLE_EARG 1

static const double TWO_PI = 6.283185307179586476925286766559;

/* W_n[m] = exp(-2*pi*i*m/n) for 0 <= m < n. Quarter turns are set exactly. */
static void make_twiddles(int n, double* re, double* im)
{
    for (int m = 0; m < n; ++m) {
        if ((4 * m) % n == 0) {
            switch ((4 * m) / n) {
            case 0: re[m] = 1.0;  im[m] = 0.0;  break;
            case 1: re[m] = 0.0;  im[m] = -1.0; break;
            case 2: re[m] = -1.0; im[m] = 0.0;  break;
            default: re[m] = 0.0; im[m] = 1.0;  break;
            }
        } else {
            double a = TWO_PI * (double)m / (double)n;
            re[m] = cos(a);
            im[m] = -sin(a);
#if ORACLE_MUTATION == 1
            im[m] = sin(a); /* mutation: inverse-transform sign */
#endif
        }
    }
}

static int check_shape(int64_t N0, int64_t N1, int n0, int n1)
{
    if (N0 < 1 || N1 < 1 || n0 < 1 || n1 < 1) return ORACLE_EARG;
    if (n0 > N0 || n1 > N1) return ORACLE_EARG;
    return ORACLE_OK;
}

/*
 * Forward transform at a list of windows.
 *   x_re, x_im : input [N0][N1], row-major; x_im may be NULL (real input).
 *   q0, q1     : window top-left corners, nwin entries; if both are NULL every
 *                window is computed in row-major (q0, q1) order and nwin must
 *                equal P0*P1.
 *   y_re, y_im : output [nwin][n0][n1], k1 fastest.
 * Returns 0, or 1 on a bad argument (nothing written).
 */
int oracle_swdft2d(const double* x_re, const double* x_im, int64_t N0, int64_t N1,
                   int32_t n0, int32_t n1, int32_t ortho,
                   const int64_t* q0, const int64_t* q1, int64_t nwin,
                   double* y_re, double* y_im)
{
    if (check_shape(N0, N1, n0, n1) != ORACLE_OK || !x_re || !y_re || !y_im || nwin < 0)
        return ORACLE_EARG;
    const int64_t P0 = N0 - n0 + 1, P1 = N1 - n1 + 1;
    if ((q0 == NULL) != (q1 == NULL)) return ORACLE_EARG;
    if (q0 == NULL && nwin != P0 * P1) return ORACLE_EARG;
    if (q0 != NULL) {
        for (int64_t w = 0; w < nwin; ++w)
            if (q0[w] < 0 || q0[w] >= P0 || q1[w] < 0 || q1[w] >= P1) return ORACLE_EARG;
    }

    double* w0r = (double*)malloc(sizeof(double) * (size_t)n0);
    double* w0i = (double*)malloc(sizeof(double) * (size_t)n0);
    double* w1r = (double*)malloc(sizeof(double) * (size_t)n1);
    double* w1i = (double*)malloc(sizeof(double) * (size_t)n1);
    if (!w0r || !w0i || !w1r || !w1i) { free(w0r); free(w0i); free(w1r); free(w1i); return ORACLE_EARG; }
    make_twiddles(n0, w0r, w0i);
    make_twiddles(n1, w1r, w1i);
    const double scale = ortho ? 1.0 / sqrt((double)n0 * (double)n1) : 1.0;

    int64_t j1_end = n1;
#if ORACLE_MUTATION == 2
    j1_end = n1 - 1; /* mutation: last column of every window dropped */
#endif

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t w = 0; w < nwin; ++w) {
        const int64_t a0 = q0 ? q0[w] : w / P1;
        const int64_t a1 = q1 ? q1[w] : w % P1;
        double* yr = y_re + w * (int64_t)n0 * n1;
        double* yi = y_im + w * (int64_t)n0 * n1;
        for (int k0 = 0; k0 < n0; ++k0) {
            for (int k1 = 0; k1 < n1; ++k1) {
                double acc_r = 0.0, acc_i = 0.0;
                for (int j0 = 0; j0 < n0; ++j0) {
                    for (int64_t j1 = 0; j1 < j1_end; ++j1) {
                        int64_t r = a0 + j0, c = a1 + j1;
#if ORACLE_MUTATION == 3
                        r = a0 + j1 % n0; c = a1 + j0 % n1; /* mutation: window transposed */
#endif
#if ORACLE_MUTATION == 4
                        c = a1 + j1 + (a1 + j1 + 1 < N1 ? 1 : 0); /* mutation: off-by-one column */
#endif
                        const double xr = x_re[r * N1 + c];
                        const double xi = x_im ? x_im[r * N1 + c] : 0.0;
                        int e0 = (int)(((int64_t)j0 * k0) % n0);
                        int e1 = (int)((j1 * k1) % n1);
#if ORACLE_MUTATION == 5
                        e0 = (int)(((int64_t)j0 * k1) % n0); /* mutation: k0 and k1 swapped */
                        e1 = (int)((j1 * k0) % n1);
#endif
                        /* t = W0[e0] * W1[e1] */
                        const double tr = w0r[e0] * w1r[e1] - w0i[e0] * w1i[e1];
                        const double ti = w0r[e0] * w1i[e1] + w0i[e0] * w1r[e1];
                        acc_r += xr * tr - xi * ti;
                        acc_i += xr * ti + xi * tr;
                    }
                }
                yr[k0 * n1 + k1] = acc_r * scale;
                yi[k0 * n1 + k1] = acc_i * scale;
            }
        }
    }
    free(w0r); free(w0i); free(w1r); free(w1i);
    return ORACLE_OK;
}

/*
 * Adjoint (conjugate transpose) of the forward map, at a list of pixels.
 *   dy_re, dy_im : cotangent [P0][P1][n0][n1], k1 fastest (all windows).
 *   r, c         : pixel coordinates, npix entries; if both are NULL every
 *                  pixel is computed in row-major order and npix = N0*N1.
 *   dx_re, dx_im : output [npix] (complex; a real input takes dx_re).
 */
int oracle_swdft2d_adjoint(const double* dy_re, const double* dy_im, int64_t N0, int64_t N1,
                           int32_t n0, int32_t n1, int32_t ortho,
                           const int64_t* r, const int64_t* c, int64_t npix,
                           double* dx_re, double* dx_im)
{
    if (check_shape(N0, N1, n0, n1) != ORACLE_OK || !dy_re || !dy_im || !dx_re || !dx_im || npix < 0)
        return ORACLE_EARG;
    if ((r == NULL) != (c == NULL)) return ORACLE_EARG;
    if (r == NULL && npix != N0 * N1) return ORACLE_EARG;
    if (r != NULL) {
        for (int64_t t = 0; t < npix; ++t)
            if (r[t] < 0 || r[t] >= N0 || c[t] < 0 || c[t] >= N1) return ORACLE_EARG;
    }
    const int64_t P0 = N0 - n0 + 1, P1 = N1 - n1 + 1;

    double* w0r = (double*)malloc(sizeof(double) * (size_t)n0);
    double* w0i = (double*)malloc(sizeof(double) * (size_t)n0);
    double* w1r = (double*)malloc(sizeof(double) * (size_t)n1);
    double* w1i = (double*)malloc(sizeof(double) * (size_t)n1);
    if (!w0r || !w0i || !w1r || !w1i) { free(w0r); free(w0i); free(w1r); free(w1i); return ORACLE_EARG; }
    make_twiddles(n0, w0r, w0i);
    make_twiddles(n1, w1r, w1i);
    const double scale = ortho ? 1.0 / sqrt((double)n0 * (double)n1) : 1.0;
    double conj_sign = -1.0;
#if ORACLE_MUTATION == 6
    conj_sign = 1.0; /* mutation: conjugate forgotten */
#endif
    int64_t first_shift = 0;
#if ORACLE_MUTATION == 7
    first_shift = 1; /* mutation: window range off by one */
#endif

#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < npix; ++t) {
        const int64_t pr = r ? r[t] : t / N1;
        const int64_t pc = c ? c[t] : t % N1;
        /* windows (q0,q1) with q0 <= pr <= q0+n0-1 and 0 <= q0 < P0, likewise q1 */
        int64_t q0_lo = pr - n0 + 1 + first_shift; if (q0_lo < 0) q0_lo = 0;
        int64_t q0_hi = pr; if (q0_hi > P0 - 1) q0_hi = P0 - 1;
        int64_t q1_lo = pc - n1 + 1; if (q1_lo < 0) q1_lo = 0;
        int64_t q1_hi = pc; if (q1_hi > P1 - 1) q1_hi = P1 - 1;
        double acc_r = 0.0, acc_i = 0.0;
        for (int64_t a0 = q0_lo; a0 <= q0_hi; ++a0) {
            for (int64_t a1 = q1_lo; a1 <= q1_hi; ++a1) {
                const int64_t j0 = pr - a0, j1 = pc - a1;
                const double* gr = dy_re + (a0 * P1 + a1) * (int64_t)n0 * n1;
                const double* gi = dy_im + (a0 * P1 + a1) * (int64_t)n0 * n1;
                for (int k0 = 0; k0 < n0; ++k0) {
                    for (int k1 = 0; k1 < n1; ++k1) {
                        const int e0 = (int)((j0 * k0) % n0);
                        const int e1 = (int)((j1 * k1) % n1);
                        const double tr = w0r[e0] * w1r[e1] - w0i[e0] * w1i[e1];
                        const double ti = conj_sign * (w0r[e0] * w1i[e1] + w0i[e0] * w1r[e1]);
                        const double ar = gr[k0 * n1 + k1], ai = gi[k0 * n1 + k1];
                        acc_r += ar * tr - ai * ti;
                        acc_i += ar * ti + ai * tr;
                    }
                }
            }
        }
        dx_re[t] = acc_r * scale;
        dx_im[t] = acc_i * scale;
    }
    free(w0r); free(w0i); free(w1r); free(w1i);
    return ORACLE_OK;
}

/*
 * Forward 3D SWDFT at a list of windows: the k-dimensional extension of
 * Sec. 4.4 (Eq. (7) and its three-dimensional instances), whose trees end in
 * the plain 3D DFT of every window:
 *
 *   a[q0][q1][q2][k0][k1][k2] = s * sum_{j0<n0} sum_{j1<n1} sum_{j2<n2}
 *        x[q0+j0][q1+j1][q2+j2] * W0[(j0 k0) mod n0] * W1[(j1 k1) mod n1] * W2[(j2 k2) mod n2]
 *
 * with s = 1, or 1/sqrt(n0 n1 n2) (the 3D analogue of the scale of Eq. (2)).
 *   x_re, x_im : input [N0][N1][N2], row-major; x_im may be NULL (real input).
 *   q0, q1, q2 : window corners, nwin entries; all NULL for every window in
 *                row-major (q0, q1, q2) order (nwin = P0*P1*P2).
 *   y_re, y_im : output [nwin][n0][n1][n2], k2 fastest.
 * Returns 0, or 1 on a bad argument (nothing written).
 */
int oracle_swdft3d(const double* x_re, const double* x_im, int64_t N0, int64_t N1, int64_t N2,
                   int32_t n0, int32_t n1, int32_t n2, int32_t ortho,
                   const int64_t* q0, const int64_t* q1, const int64_t* q2, int64_t nwin,
                   double* y_re, double* y_im)
{
    if (check_shape(N0, N1, n0, n1) != ORACLE_OK || N2 < 1 || n2 < 1 || n2 > N2 || !x_re ||
        !y_re || !y_im || nwin < 0)
        return ORACLE_EARG;
    const int64_t P0 = N0 - n0 + 1, P1 = N1 - n1 + 1, P2 = N2 - n2 + 1;
    const int given = (q0 != NULL) + (q1 != NULL) + (q2 != NULL);
    if (given != 0 && given != 3) return ORACLE_EARG;
    if (given == 0 && nwin != P0 * P1 * P2) return ORACLE_EARG;
    if (given == 3) {
        for (int64_t w = 0; w < nwin; ++w)
            if (q0[w] < 0 || q0[w] >= P0 || q1[w] < 0 || q1[w] >= P1 || q2[w] < 0 || q2[w] >= P2)
                return ORACLE_EARG;
    }

    double* w0r = (double*)malloc(sizeof(double) * (size_t)n0);
    double* w0i = (double*)malloc(sizeof(double) * (size_t)n0);
    double* w1r = (double*)malloc(sizeof(double) * (size_t)n1);
    double* w1i = (double*)malloc(sizeof(double) * (size_t)n1);
    double* w2r = (double*)malloc(sizeof(double) * (size_t)n2);
    double* w2i = (double*)malloc(sizeof(double) * (size_t)n2);
    if (!w0r || !w0i || !w1r || !w1i || !w2r || !w2i) {
        free(w0r); free(w0i); free(w1r); free(w1i); free(w2r); free(w2i);
        return ORACLE_EARG;
    }
    make_twiddles(n0, w0r, w0i);
    make_twiddles(n1, w1r, w1i);
    make_twiddles(n2, w2r, w2i);
#if ORACLE_MUTATION == 10
    if (n1 <= n2) make_twiddles(n1, w2r, w2i); /* mutation: axis-2 roots of length n1 */
#endif
    const double scale = ortho ? 1.0 / sqrt((double)n0 * (double)n1 * (double)n2) : 1.0;
    int64_t j2_end = n2;
#if ORACLE_MUTATION == 8
    j2_end = n2 - 1; /* mutation: last slice of every window dropped */
#endif
    const int64_t nk = (int64_t)n0 * n1 * n2;

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t w = 0; w < nwin; ++w) {
        const int64_t a0 = q0 ? q0[w] : w / (P1 * P2);
        const int64_t a1 = q1 ? q1[w] : (w / P2) % P1;
        const int64_t a2 = q2 ? q2[w] : w % P2;
        double* yr = y_re + w * nk;
        double* yi = y_im + w * nk;
        for (int k0 = 0; k0 < n0; ++k0) {
            for (int k1 = 0; k1 < n1; ++k1) {
                for (int k2 = 0; k2 < n2; ++k2) {
                    double acc_r = 0.0, acc_i = 0.0;
                    for (int j0 = 0; j0 < n0; ++j0) {
                        for (int j1 = 0; j1 < n1; ++j1) {
                            for (int64_t j2 = 0; j2 < j2_end; ++j2) {
                                const int64_t idx = ((a0 + j0) * N1 + (a1 + j1)) * N2 + (a2 + j2);
                                const double xr = x_re[idx];
                                const double xi = x_im ? x_im[idx] : 0.0;
                                const int e0 = (int)(((int64_t)j0 * k0) % n0);
                                int e1 = (int)(((int64_t)j1 * k1) % n1);
                                int e2 = (int)((j2 * k2) % n2);
#if ORACLE_MUTATION == 9
                                e1 = (int)(((int64_t)j1 * k2) % n1); /* mutation: k1 and k2 swapped */
                                e2 = (int)((j2 * k1) % n2);
#endif
                                /* t = W0[e0] * W1[e1] * W2[e2] */
                                const double ur = w0r[e0] * w1r[e1] - w0i[e0] * w1i[e1];
                                const double ui = w0r[e0] * w1i[e1] + w0i[e0] * w1r[e1];
                                const double tr = ur * w2r[e2] - ui * w2i[e2];
                                const double ti = ur * w2i[e2] + ui * w2r[e2];
                                acc_r += xr * tr - xi * ti;
                                acc_i += xr * ti + xi * tr;
                            }
                        }
                    }
                    yr[((int64_t)k0 * n1 + k1) * n2 + k2] = acc_r * scale;
                    yi[((int64_t)k0 * n1 + k1) * n2 + k2] = acc_i * scale;
                }
            }
        }
    }
    free(w0r); free(w0i); free(w1r); free(w1i); free(w2r); free(w2i);
    return ORACLE_OK;
}

/*
 * Adjoint (conjugate transpose) of the 3D forward map above, at a list of
 * voxels:
 *
 *   dx[r0][r1][r2] = s * sum over windows (q0,q1,q2) covering the voxel of
 *        sum_{k0,k1,k2} dy[q0][q1][q2][k0][k1][k2]
 *        * conj(W0[((r0-q0) k0) mod n0] * W1[((r1-q1) k1) mod n1] * W2[((r2-q2) k2) mod n2])
 *
 *   dy_re, dy_im : cotangent [P0][P1][P2][n0][n1][n2], k2 fastest (all windows).
 *   v0, v1, v2   : voxel coordinates, nvox entries; all NULL for every voxel in
 *                  row-major order (nvox = N0*N1*N2).
 *   dx_re, dx_im : output [nvox] (complex; a real input takes dx_re).
 */
int oracle_swdft3d_adjoint(const double* dy_re, const double* dy_im, int64_t N0, int64_t N1,
                           int64_t N2, int32_t n0, int32_t n1, int32_t n2, int32_t ortho,
                           const int64_t* v0, const int64_t* v1, const int64_t* v2, int64_t nvox,
                           double* dx_re, double* dx_im)
{
    if (check_shape(N0, N1, n0, n1) != ORACLE_OK || N2 < 1 || n2 < 1 || n2 > N2 || !dy_re ||
        !dy_im || !dx_re || !dx_im || nvox < 0)
        return ORACLE_EARG;
    const int given = (v0 != NULL) + (v1 != NULL) + (v2 != NULL);
    if (given != 0 && given != 3) return ORACLE_EARG;
    if (given == 0 && nvox != N0 * N1 * N2) return ORACLE_EARG;
    if (given == 3) {
        for (int64_t t = 0; t < nvox; ++t)
            if (v0[t] < 0 || v0[t] >= N0 || v1[t] < 0 || v1[t] >= N1 || v2[t] < 0 || v2[t] >= N2)
                return ORACLE_EARG;
    }
    const int64_t P0 = N0 - n0 + 1, P1 = N1 - n1 + 1, P2 = N2 - n2 + 1;

    double* w0r = (double*)malloc(sizeof(double) * (size_t)n0);
    double* w0i = (double*)malloc(sizeof(double) * (size_t)n0);
    double* w1r = (double*)malloc(sizeof(double) * (size_t)n1);
    double* w1i = (double*)malloc(sizeof(double) * (size_t)n1);
    double* w2r = (double*)malloc(sizeof(double) * (size_t)n2);
    double* w2i = (double*)malloc(sizeof(double) * (size_t)n2);
    if (!w0r || !w0i || !w1r || !w1i || !w2r || !w2i) {
        free(w0r); free(w0i); free(w1r); free(w1i); free(w2r); free(w2i);
        return ORACLE_EARG;
    }
    make_twiddles(n0, w0r, w0i);
    make_twiddles(n1, w1r, w1i);
    make_twiddles(n2, w2r, w2i);
    const double scale = ortho ? 1.0 / sqrt((double)n0 * (double)n1 * (double)n2) : 1.0;
    double conj_sign = -1.0;
#if ORACLE_MUTATION == 11
    conj_sign = 1.0; /* mutation: conjugate forgotten */
#endif
    int64_t shift1 = 0;
#if ORACLE_MUTATION == 12
    shift1 = 1; /* mutation: axis-1 window range off by one */
#endif
    const int64_t nk = (int64_t)n0 * n1 * n2;

#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < nvox; ++t) {
        const int64_t r0 = v0 ? v0[t] : t / (N1 * N2);
        const int64_t r1 = v1 ? v1[t] : (t / N2) % N1;
        const int64_t r2 = v2 ? v2[t] : t % N2;
        /* windows with q_i <= r_i <= q_i + n_i - 1 and 0 <= q_i < P_i */
        int64_t lo0 = r0 - n0 + 1; if (lo0 < 0) lo0 = 0;
        int64_t hi0 = r0; if (hi0 > P0 - 1) hi0 = P0 - 1;
        int64_t lo1 = r1 - n1 + 1 + shift1; if (lo1 < 0) lo1 = 0;
        int64_t hi1 = r1; if (hi1 > P1 - 1) hi1 = P1 - 1;
        int64_t lo2 = r2 - n2 + 1; if (lo2 < 0) lo2 = 0;
        int64_t hi2 = r2; if (hi2 > P2 - 1) hi2 = P2 - 1;
        double acc_r = 0.0, acc_i = 0.0;
        for (int64_t a0 = lo0; a0 <= hi0; ++a0) {
            for (int64_t a1 = lo1; a1 <= hi1; ++a1) {
                for (int64_t a2 = lo2; a2 <= hi2; ++a2) {
                    const int64_t j0 = r0 - a0, j1 = r1 - a1, j2 = r2 - a2;
                    const int64_t base = ((a0 * P1 + a1) * P2 + a2) * nk;
                    for (int k0 = 0; k0 < n0; ++k0) {
                        for (int k1 = 0; k1 < n1; ++k1) {
                            for (int k2 = 0; k2 < n2; ++k2) {
                                const int e0 = (int)((j0 * k0) % n0);
                                const int e1 = (int)((j1 * k1) % n1);
                                const int e2 = (int)((j2 * k2) % n2);
                                /* u = W0[e0] W1[e1], t = conj(u W2[e2]) */
                                const double ur = w0r[e0] * w1r[e1] - w0i[e0] * w1i[e1];
                                const double ui = w0r[e0] * w1i[e1] + w0i[e0] * w1r[e1];
                                const double tr = ur * w2r[e2] - ui * w2i[e2];
                                const double ti = conj_sign * (ur * w2i[e2] + ui * w2r[e2]);
                                const int64_t idx = base + ((int64_t)k0 * n1 + k1) * n2 + k2;
                                const double gr = dy_re[idx], gi = dy_im[idx];
                                acc_r += gr * tr - gi * ti;
                                acc_i += gr * ti + gi * tr;
                            }
                        }
                    }
                }
            }
        }
        dx_re[t] = acc_r * scale;
        dx_im[t] = acc_i * scale;
    }
    free(w0r); free(w0i); free(w1r); free(w1i); free(w2r); free(w2i);
    return ORACLE_OK;
}

/* Number of threads an OpenMP region of this library would use (1 if built
 * without OpenMP). Reported beside timings of the oracle. */
#ifdef _OPENMP
#include <omp.h>
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_threads(int n) { if (n >= 1) omp_set_num_threads(n); }
#else
int oracle_num_threads(void) { return 1; }
void oracle_set_threads(int n) { (void)n; }
#endif
