"""Pins that tie the FP64 oracle to facts fixed by the mathematics, not to itself.

Each pin takes an ``oracle.Oracle`` and raises AssertionError when the oracle
disagrees with:
  * an independent formulation (the factorised matrix form F0 X F1^T of
    Eq. (3)-(4), built with numpy; numpy.fft.fft2 on each window, also for
    windows of 3, 6, 9, 12 and 24),
  * exact Gaussian-integer brute force for n_i <= 4 (all twiddles are
    powers of -i there, so every sum is exact),
  * closed forms (impulse, constant, on-bin exponential and cosine),
  * invariants (Parseval per window, the shift theorem between neighbouring
    windows that recursive sliding DFTs are built on (Sec. 2), linearity),
  * the adjoint identities (dot-product test, exact central differences of a
    quadratic loss),
  * for the 3D extension (Sec. 4.4): numpy.fft.fftn per window, separable
    inputs against 1D sliding DFTs, exact Gaussian integers, the sliding
    recurrence along the last axis, Parseval and the orthonormal scale.

``ALL_PINS`` lists them so the mutation test can run every pin against
deliberately broken builds of the oracle.
"""
from __future__ import annotations

import numpy as np

import workloads


def _dft_matrix(n: int) -> np.ndarray:
    k = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(k, k) / n)


def _rel(a, b) -> float:
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def pin_matrix_form(orc):
    """y_w = F_n0 X_w F_n1^T for every window (factorisation, Eq. (3)-(4))."""
    rng = np.random.default_rng(11)
    for (N0, N1, n0, n1) in [(7, 9, 4, 8), (9, 6, 8, 2), (5, 11, 1, 4), (6, 6, 2, 2), (8, 5, 8, 1)]:
        x = rng.standard_normal((N0, N1)) + 1j * rng.standard_normal((N0, N1))
        y = orc.swdft2d(x, n0, n1)
        F0, F1 = _dft_matrix(n0), _dft_matrix(n1)
        for q0 in range(N0 - n0 + 1):
            for q1 in range(N1 - n1 + 1):
                ref = F0 @ x[q0:q0 + n0, q1:q1 + n1] @ F1.T
                assert _rel(y[q0, q1], ref) < 1e-13, (N0, N1, n0, n1, q0, q1)


def pin_fft2(orc):
    """Each window equals numpy.fft.fft2 of that window (real and complex x)."""
    rng = np.random.default_rng(12)
    for (N0, N1, n0, n1) in [(20, 17, 8, 4), (16, 16, 16, 16), (12, 40, 4, 32)]:
        for cplx in (False, True):
            x = rng.standard_normal((N0, N1))
            if cplx:
                x = x + 1j * rng.standard_normal((N0, N1))
            y = orc.swdft2d(x, n0, n1)
            P0, P1 = N0 - n0 + 1, N1 - n1 + 1
            win = np.lib.stride_tricks.sliding_window_view(x, (n0, n1))
            ref = np.fft.fft2(win, axes=(-2, -1))
            assert y.shape == (P0, P1, n0, n1)
            assert _rel(y, ref) < 1e-13, (N0, N1, n0, n1, cplx)


def pin_mixed_radix(orc):
    """Windows that are not powers of two (the radix-3 and mixed 2/3 trees of
    Sec. 5): each window equals numpy.fft.fft2 of that window, the twiddle of
    a third of a turn is exp(-2 pi i / 3) (checked through an on-bin
    exponential), and Parseval holds per window."""
    rng = np.random.default_rng(14)
    for (N0, N1, n0, n1) in [(9, 14, 3, 6), (20, 15, 12, 9), (30, 7, 24, 3), (13, 27, 6, 12)]:
        x = rng.standard_normal((N0, N1)) + 1j * rng.standard_normal((N0, N1))
        y = orc.swdft2d(x, n0, n1)
        win = np.lib.stride_tricks.sliding_window_view(x, (n0, n1))
        assert _rel(y, np.fft.fft2(win, axes=(-2, -1))) < 1e-13, (N0, N1, n0, n1)
        energy = np.sum(np.abs(win) ** 2, axis=(-2, -1))
        assert np.allclose(np.sum(np.abs(y) ** 2, axis=(-2, -1)), n0 * n1 * energy, rtol=1e-12)
    # x = exp(2 pi i (k0 r / 3 + k1 c / 6)): every window is on bin (k0, k1) with
    # value n0 n1 times the phase of its corner, all other bins zero
    N0, N1, n0, n1, k0, k1 = 8, 11, 3, 6, 1, 5
    r, c = np.meshgrid(np.arange(N0), np.arange(N1), indexing="ij")
    x = np.exp(2j * np.pi * (k0 * r / n0 + k1 * c / n1))
    y = orc.swdft2d(x, n0, n1)
    P0, P1 = N0 - n0 + 1, N1 - n1 + 1
    q0, q1 = np.meshgrid(np.arange(P0), np.arange(P1), indexing="ij")
    corner = np.exp(2j * np.pi * (k0 * q0 / n0 + k1 * q1 / n1))
    assert np.allclose(y[:, :, k0, k1], n0 * n1 * corner, atol=1e-12)
    y[:, :, k0, k1] = 0
    assert np.max(np.abs(y)) < 1e-12


def pin_whole_array(orc):
    """N = n: one window, the textbook 2D DFT of the whole array."""
    rng = np.random.default_rng(13)
    x = rng.standard_normal((8, 32))
    y = orc.swdft2d(x, 8, 32)
    assert y.shape == (1, 1, 8, 32)
    assert _rel(y[0, 0], np.fft.fft2(x)) < 1e-13


def pin_exact_small(orc):
    """Gaussian-integer brute force, exact, on the 2 x 5 array with 2 x 4
    windows of the worked example of Fig. 3 and a few more tiny shapes.

    For n <= 4 the twiddles are exactly (-i)^(4m/n), so integer inputs give
    integer outputs and the oracle must match them bit for bit.
    """
    rng = np.random.default_rng(14)
    for (N0, N1, n0, n1) in [(2, 5, 2, 4), (4, 4, 4, 4), (3, 6, 1, 2), (5, 3, 4, 1)]:
        xr = rng.integers(-9, 10, size=(N0, N1))
        xi = rng.integers(-9, 10, size=(N0, N1))
        x = xr + 1j * xi
        y = orc.swdft2d(x.astype(np.complex128), n0, n1)
        for q0 in range(N0 - n0 + 1):
            for q1 in range(N1 - n1 + 1):
                for k0 in range(n0):
                    for k1 in range(n1):
                        acc_r = 0
                        acc_i = 0
                        for j0 in range(n0):
                            for j1 in range(n1):
                                # exponent of -i: quarter turns of W0^(j0 k0) W1^(j1 k1)
                                e = ((4 // n0) * j0 * k0 if n0 > 1 else 0) + \
                                    ((4 // n1) * j1 * k1 if n1 > 1 else 0)
                                a, b = int(xr[q0 + j0, q1 + j1]), int(xi[q0 + j0, q1 + j1])
                                for _ in range(e % 4):  # multiply by -i
                                    a, b = b, -a
                                acc_r += a
                                acc_i += b
                        got = y[q0, q1, k0, k1]
                        assert got.real == acc_r and got.imag == acc_i, \
                            (N0, N1, n0, n1, q0, q1, k0, k1, got, acc_r, acc_i)


def pin_impulse(orc):
    """x = delta at (r, c): windows that contain it give the unit-modulus
    phase exp(-2 pi i ((r-q0) k0/n0 + (c-q1) k1/n1)), other windows give 0."""
    N0, N1, n0, n1 = 12, 14, 4, 8
    r, c = 5, 9
    x = np.zeros((N0, N1))
    x[r, c] = 1.0
    y = orc.swdft2d(x, n0, n1)
    k0 = np.arange(n0)[:, None]
    k1 = np.arange(n1)[None, :]
    for q0 in range(N0 - n0 + 1):
        for q1 in range(N1 - n1 + 1):
            inside = (q0 <= r < q0 + n0) and (q1 <= c < q1 + n1)
            if inside:
                ref = np.exp(-2j * np.pi * ((r - q0) * k0 / n0 + (c - q1) * k1 / n1))
                assert np.max(np.abs(y[q0, q1] - ref)) < 1e-14
                assert np.allclose(np.abs(y[q0, q1]), 1.0, atol=1e-14)
            else:
                assert np.all(y[q0, q1] == 0)


def pin_constant(orc):
    """x = C everywhere: a = C n0 n1 at k = (0,0) and exactly 0 elsewhere for
    n_i <= 4 (exact twiddles), <= 1e-13 relative for larger windows."""
    for (n0, n1, exact) in [(4, 2, True), (16, 8, False)]:
        C = 3.25
        x = np.full((n0 + 5, n1 + 3), C)
        y = orc.swdft2d(x, n0, n1)
        expect = np.zeros((n0, n1), complex)
        expect[0, 0] = C * n0 * n1
        for q0 in range(y.shape[0]):
            for q1 in range(y.shape[1]):
                if exact:
                    assert np.array_equal(y[q0, q1], expect)
                else:
                    assert np.max(np.abs(y[q0, q1] - expect)) < 1e-13 * C * n0 * n1


def pin_onbin_exponential(orc):
    """x[r][c] = exp(2 pi i (f0 r/n0 + f1 c/n1)): a single bin k = (f0, f1)
    holding n0 n1 exp(2 pi i (f0 q0/n0 + f1 q1/n1)); every other bin is 0."""
    N0, N1, n0, n1 = 19, 23, 8, 16
    f0, f1 = 3, 11
    r = np.arange(N0)[:, None]
    c = np.arange(N1)[None, :]
    x = np.exp(2j * np.pi * (f0 * r / n0 + f1 * c / n1))
    y = orc.swdft2d(x, n0, n1)
    q0 = np.arange(N0 - n0 + 1)[:, None]
    q1 = np.arange(N1 - n1 + 1)[None, :]
    peak = n0 * n1 * np.exp(2j * np.pi * (f0 * q0 / n0 + f1 * q1 / n1))
    assert np.max(np.abs(y[:, :, f0, f1] - peak)) < 1e-11
    rest = y.copy()
    rest[:, :, f0, f1] = 0
    assert np.max(np.abs(rest)) < 1e-11


def pin_onbin_cosine(orc):
    """Real cosine 5 cos(2 pi (f0 r/N0 + f1 c/N1) + phi) with on-bin
    frequencies (as in the planted workload): two bins of half amplitude,
    k = (k0, k1) and its mirror (-k0, -k1), each of magnitude 5 n0 n1 / 2."""
    N0, N1, n0, n1 = 64, 48, 16, 8
    k0, k1, ph = 3, 2, 0.7
    f0, f1 = k0 * N0 // n0, k1 * N1 // n1
    r = np.arange(N0)[:, None]
    c = np.arange(N1)[None, :]
    x = 5.0 * np.cos(2 * np.pi * (f0 * r / N0 + f1 * c / N1) + ph)
    y = orc.swdft2d(x, n0, n1, windows=workloads.window_sample(N0 - n0 + 1, N1 - n1 + 1, 40, 3))
    mag = np.abs(y)
    assert np.allclose(mag[:, k0, k1], 5 * n0 * n1 / 2, rtol=1e-12)
    assert np.allclose(mag[:, (-k0) % n0, (-k1) % n1], 5 * n0 * n1 / 2, rtol=1e-12)
    mag[:, k0, k1] = 0
    mag[:, (-k0) % n0, (-k1) % n1] = 0
    assert np.max(mag) < 1e-10


def pin_parseval(orc):
    """Per window: sum_k |a_k|^2 = n0 n1 sum_j |x_j|^2; with the orthonormal
    scale of Eq. (2) the two sides are equal."""
    rng = np.random.default_rng(15)
    N0, N1, n0, n1 = 21, 18, 8, 4
    x = rng.standard_normal((N0, N1)) + 1j * rng.standard_normal((N0, N1))
    win = np.lib.stride_tricks.sliding_window_view(x, (n0, n1))
    energy = np.sum(np.abs(win) ** 2, axis=(-2, -1))
    y = orc.swdft2d(x, n0, n1)
    assert np.allclose(np.sum(np.abs(y) ** 2, axis=(-2, -1)), n0 * n1 * energy, rtol=1e-12)
    yo = orc.swdft2d(x, n0, n1, norm="ortho")
    assert np.allclose(np.sum(np.abs(yo) ** 2, axis=(-2, -1)), energy, rtol=1e-12)
    # n0 n1 = 32 is not a square, so compare the scale itself
    assert np.allclose(y, yo * np.sqrt(n0 * n1), rtol=1e-13, atol=1e-13)


def pin_shift_theorem(orc):
    """Neighbouring windows: sliding one column right replaces column q1 by
    column q1+n1 (Fig. 3) and rotates by W1^{-k1}:
        a[q0][q1+1][k] = W1^{-k1} (a[q0][q1][k] + sum_j0 W0^{j0 k0}
                         (x[q0+j0][q1+n1] - x[q0+j0][q1]))
    and likewise for a step down one row."""
    rng = np.random.default_rng(16)
    N0, N1, n0, n1 = 13, 15, 4, 8
    x = rng.standard_normal((N0, N1)) + 1j * rng.standard_normal((N0, N1))
    y = orc.swdft2d(x, n0, n1)
    F0, F1 = _dft_matrix(n0), _dft_matrix(n1)
    k0 = np.arange(n0)[:, None]
    k1 = np.arange(n1)[None, :]
    rot1 = np.exp(2j * np.pi * k1 / n1)
    rot0 = np.exp(2j * np.pi * k0 / n0)
    for q0 in range(N0 - n0 + 1):
        for q1 in range(N1 - n1):
            diff = F0 @ (x[q0:q0 + n0, q1 + n1] - x[q0:q0 + n0, q1])
            pred = rot1 * (y[q0, q1] + diff[:, None])
            assert np.max(np.abs(y[q0, q1 + 1] - pred)) < 1e-11
    for q0 in range(N0 - n0):
        for q1 in range(N1 - n1 + 1):
            diff = F1 @ (x[q0 + n0, q1:q1 + n1] - x[q0, q1:q1 + n1])
            pred = rot0 * (y[q0, q1] + diff[None, :])
            assert np.max(np.abs(y[q0 + 1, q1] - pred)) < 1e-11


def pin_linearity_and_sampling(orc):
    """Linearity in x; sampled windows equal the same entries of the full output."""
    rng = np.random.default_rng(17)
    N0, N1, n0, n1 = 17, 20, 8, 8
    a = rng.standard_normal((N0, N1))
    b = rng.standard_normal((N0, N1)) + 1j * rng.standard_normal((N0, N1))
    ya, yb = orc.swdft2d(a, n0, n1), orc.swdft2d(b, n0, n1)
    yab = orc.swdft2d(2.5 * a - 1.5j * b, n0, n1)
    assert _rel(yab, 2.5 * ya - 1.5j * yb) < 1e-13
    q0, q1 = workloads.window_sample(N0 - n0 + 1, N1 - n1 + 1, 25, 5)
    ys = orc.swdft2d(b, n0, n1, windows=(q0, q1))
    assert np.array_equal(ys, yb[q0, q1])


def pin_adjoint_dot(orc):
    """<M x, g> = <x, M^H g> for random complex x, g (several shapes)."""
    rng = np.random.default_rng(18)
    for (N0, N1, n0, n1) in [(11, 13, 4, 8), (9, 9, 8, 2), (6, 10, 1, 4)]:
        x = rng.standard_normal((N0, N1)) + 1j * rng.standard_normal((N0, N1))
        g = rng.standard_normal((N0 - n0 + 1, N1 - n1 + 1, n0, n1)) + \
            1j * rng.standard_normal((N0 - n0 + 1, N1 - n1 + 1, n0, n1))
        lhs = np.vdot(g, orc.swdft2d(x, n0, n1))
        rhs = np.vdot(orc.swdft2d_adjoint(g, N0, N1), x)
        assert abs(lhs - rhs) < 1e-11 * max(abs(lhs), 1.0), (N0, N1, n0, n1)
        # ortho scale too
        lhs = np.vdot(g, orc.swdft2d(x, n0, n1, norm="ortho"))
        rhs = np.vdot(orc.swdft2d_adjoint(g, N0, N1, norm="ortho"), x)
        assert abs(lhs - rhs) < 1e-11 * max(abs(lhs), 1.0)


def pin_adjoint_sampled(orc):
    """Sampled adjoint pixels equal the same entries of the full adjoint."""
    rng = np.random.default_rng(19)
    N0, N1, n0, n1 = 14, 12, 4, 4
    g = rng.standard_normal((N0 - n0 + 1, N1 - n1 + 1, n0, n1)) + 0j
    full = orc.swdft2d_adjoint(g, N0, N1)
    r, c = workloads.pixel_sample(N0, N1, 30, 2)
    assert np.array_equal(orc.swdft2d_adjoint(g, N0, N1, pixels=(r, c)), full[r, c])


def pin_quadratic_fd(orc):
    """L(x) = sum w |M x|^2 is quadratic, so the central difference with h = 1
    is exact up to rounding and must equal Re(M^H (2 w M x)) for real x."""
    rng = np.random.default_rng(20)
    N0, N1, n0, n1 = 10, 12, 4, 4
    x = rng.standard_normal((N0, N1))
    w = (rng.random((n0, n1)) < 0.4).astype(float)
    w[0, 1] = 1.0

    def loss(z):
        return float(np.sum(w * np.abs(orc.swdft2d(z, n0, n1)) ** 2))

    grad = orc.swdft2d_adjoint(2.0 * w * orc.swdft2d(x, n0, n1), N0, N1).real
    for (r, c) in [(0, 0), (N0 - 1, N1 - 1), (3, 7), (0, N1 - 1), (5, 0)]:
        e = np.zeros_like(x)
        e[r, c] = 1.0
        fd = (loss(x + e) - loss(x - e)) / 2.0
        assert abs(fd - grad[r, c]) < 1e-10 * max(1.0, abs(fd)), (r, c, fd, grad[r, c])


# ---- 3D SWDFT (the k-dimensional extension of Sec. 4.4, k = 3)

def pin3d_fftn(orc):
    """Each 3D window equals numpy.fft.fftn of that window (real and complex
    x; unequal window sides so axes cannot be confused; whole-array window)."""
    rng = np.random.default_rng(31)
    for (N, n) in [((7, 9, 11), (2, 4, 8)), ((9, 8, 6), (8, 1, 4)), ((5, 6, 7), (1, 4, 2)),
                   ((6, 7, 8), (4, 4, 4)), ((4, 8, 2), (4, 8, 2))]:
        for cplx in (False, True):
            x = rng.standard_normal(N)
            if cplx:
                x = x + 1j * rng.standard_normal(N)
            y = orc.swdft3d(x, *n)
            win = np.lib.stride_tricks.sliding_window_view(x, n)
            ref = np.fft.fftn(win, axes=(-3, -2, -1))
            assert y.shape == tuple(N[i] - n[i] + 1 for i in range(3)) + tuple(n)
            assert _rel(y, ref) < 1e-13, (N, n, cplx)


def pin3d_separable(orc):
    """x = a (x) b (x) c (outer product): every window's 3D DFT is the
    product of the three 1D sliding DFTs, each taken from numpy.fft.fft."""
    rng = np.random.default_rng(32)
    (N0, N1, N2), (n0, n1, n2) = (10, 9, 12), (4, 2, 8)
    a = rng.standard_normal(N0) + 1j * rng.standard_normal(N0)
    b = rng.standard_normal(N1)
    c = rng.standard_normal(N2) + 1j * rng.standard_normal(N2)
    x = a[:, None, None] * b[None, :, None] * c[None, None, :]
    y = orc.swdft3d(x, n0, n1, n2)
    A = np.fft.fft(np.lib.stride_tricks.sliding_window_view(a, n0), axis=-1)
    B = np.fft.fft(np.lib.stride_tricks.sliding_window_view(b, n1), axis=-1)
    C = np.fft.fft(np.lib.stride_tricks.sliding_window_view(c, n2), axis=-1)
    ref = (A[:, None, None, :, None, None] * B[None, :, None, None, :, None] *
           C[None, None, :, None, None, :])
    assert _rel(y, ref) < 1e-13


def pin3d_exact_small(orc):
    """Gaussian-integer brute force, exact, with n_i <= 4 (all twiddles are
    powers of -i, so integer inputs give integer outputs bit for bit)."""
    rng = np.random.default_rng(33)
    for (N, n) in [((3, 4, 5), (2, 4, 2)), ((4, 3, 4), (4, 1, 4))]:
        xr = rng.integers(-9, 10, size=N)
        xi = rng.integers(-9, 10, size=N)
        y = orc.swdft3d((xr + 1j * xi).astype(np.complex128), *n)
        P = [N[i] - n[i] + 1 for i in range(3)]
        for q in np.ndindex(*P):
            for k in np.ndindex(*n):
                acc_r = acc_i = 0
                for j in np.ndindex(*n):
                    e = sum((4 // n[i]) * j[i] * k[i] if n[i] > 1 else 0 for i in range(3))
                    a = int(xr[q[0] + j[0], q[1] + j[1], q[2] + j[2]])
                    b = int(xi[q[0] + j[0], q[1] + j[1], q[2] + j[2]])
                    for _ in range(e % 4):  # multiply by -i
                        a, b = b, -a
                    acc_r += a
                    acc_i += b
                got = y[q + k]
                assert got.real == acc_r and got.imag == acc_i, (N, n, q, k)


def pin3d_shift_axis2(orc):
    """Sliding one step along the last axis replaces the plane j2 = 0 by the
    plane j2 = n2 and rotates by W2^{-k2}:
        a[q0][q1][q2+1][k] = W2^{-k2} (a[q0][q1][q2][k] + F01(x[.., q2+n2] - x[.., q2])[k0][k1])
    where F01 is the 2D DFT over the first two axes (numpy.fft.fft2)."""
    rng = np.random.default_rng(34)
    (N0, N1, N2), (n0, n1, n2) = (7, 8, 12), (4, 2, 8)
    x = rng.standard_normal((N0, N1, N2)) + 1j * rng.standard_normal((N0, N1, N2))
    y = orc.swdft3d(x, n0, n1, n2)
    rot = np.exp(2j * np.pi * np.arange(n2) / n2)[None, None, :]
    for q0 in range(N0 - n0 + 1):
        for q1 in range(N1 - n1 + 1):
            for q2 in range(N2 - n2):
                d = np.fft.fft2(x[q0:q0 + n0, q1:q1 + n1, q2 + n2] - x[q0:q0 + n0, q1:q1 + n1, q2])
                pred = rot * (y[q0, q1, q2] + d[:, :, None])
                assert np.max(np.abs(y[q0, q1, q2 + 1] - pred)) < 1e-11


def pin3d_parseval_ortho(orc):
    """Per window: sum_k |a_k|^2 = n0 n1 n2 sum_j |x_j|^2; the orthonormal
    scale 1/sqrt(n0 n1 n2) makes the two sides equal; sampled windows equal
    the same entries of the full output."""
    rng = np.random.default_rng(35)
    (N0, N1, N2), (n0, n1, n2) = (9, 10, 11), (4, 8, 2)
    x = rng.standard_normal((N0, N1, N2))
    win = np.lib.stride_tricks.sliding_window_view(x, (n0, n1, n2))
    energy = np.sum(np.abs(win) ** 2, axis=(-3, -2, -1))
    y = orc.swdft3d(x, n0, n1, n2)
    assert np.allclose(np.sum(np.abs(y) ** 2, axis=(-3, -2, -1)), n0 * n1 * n2 * energy, rtol=1e-12)
    yo = orc.swdft3d(x, n0, n1, n2, norm="ortho")
    assert np.allclose(np.sum(np.abs(yo) ** 2, axis=(-3, -2, -1)), energy, rtol=1e-12)
    q = (np.array([0, 5, 2, 5]), np.array([0, 2, 1, 2]), np.array([9, 0, 4, 9]))
    assert np.array_equal(orc.swdft3d(x, n0, n1, n2, windows=q), y[q])


def _forward3d_matrix(N, n):
    """The 3D forward map as an explicit matrix, built with numpy.fft.fftn of
    the windows of every unit impulse (no oracle code): column v is the
    output of the impulse at voxel v, flattened [P0][P1][P2][n0][n1][n2]."""
    cols = []
    for v in range(int(np.prod(N))):
        e = np.zeros(int(np.prod(N)))
        e[v] = 1.0
        win = np.lib.stride_tricks.sliding_window_view(e.reshape(N), n)
        cols.append(np.fft.fftn(win, axes=(-3, -2, -1)).ravel())
    return np.stack(cols, axis=1)


def pin3d_adjoint_matrix(orc):
    """The 3D adjoint equals the conjugate transpose of the explicit forward
    matrix (numpy fftn per window) on small volumes, unequal window sides,
    and with the orthonormal scale."""
    rng = np.random.default_rng(36)
    for N, n in [((4, 5, 6), (2, 4, 2)), ((5, 4, 3), (4, 1, 2)), ((3, 6, 5), (1, 2, 4))]:
        M = _forward3d_matrix(N, n)
        P = tuple(N[i] - n[i] + 1 for i in range(3))
        g = rng.standard_normal(P + n) + 1j * rng.standard_normal(P + n)
        ref = (M.conj().T @ g.ravel()).reshape(N)
        got = orc.swdft3d_adjoint(g, *N)
        assert _rel(got, ref) < 1e-13, (N, n)
        scale = 1.0 / np.sqrt(np.prod(n))
        assert _rel(orc.swdft3d_adjoint(g, *N, norm="ortho"), ref * scale) < 1e-13


def pin3d_adjoint_dot_fd(orc):
    """<M x, g> = <x, M^H g> against the 3D forward oracle; the quadratic
    loss L = sum w |M x|^2 has exact central differences (h = 1) equal to
    Re(M^H (2 w M x)) at every sampled voxel (corners included); sampled
    voxels equal the same entries of the full adjoint."""
    rng = np.random.default_rng(37)
    N, n = (7, 8, 9), (4, 2, 4)
    P = tuple(N[i] - n[i] + 1 for i in range(3))
    x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    g = rng.standard_normal(P + n) + 1j * rng.standard_normal(P + n)
    lhs = np.vdot(g, orc.swdft3d(x, *n))
    rhs = np.vdot(orc.swdft3d_adjoint(g, *N), x)
    assert abs(lhs - rhs) < 1e-11 * max(abs(lhs), 1.0)
    xr = rng.standard_normal(N)
    w = (rng.random(n) < 0.3).astype(float)
    w[0, 1, 1] = 1.0

    def loss(z):
        return float(np.sum(w * np.abs(orc.swdft3d(z, *n)) ** 2))

    grad = orc.swdft3d_adjoint(2.0 * w * orc.swdft3d(xr, *n), *N).real
    vox = [(0, 0, 0), (N[0] - 1, N[1] - 1, N[2] - 1), (3, 4, 5), (0, N[1] - 1, 2), (6, 0, 8)]
    for v in vox:
        e = np.zeros(N)
        e[v] = 1.0
        fd = (loss(xr + e) - loss(xr - e)) / 2.0
        assert abs(fd - grad[v]) < 1e-10 * max(1.0, abs(fd)), (v, fd, grad[v])
    vv = tuple(np.array(a) for a in zip(*vox))
    full = orc.swdft3d_adjoint(g, *N)
    assert np.array_equal(orc.swdft3d_adjoint(g, *N, voxels=vv), full[vv])


PINS_3D = [pin3d_fftn, pin3d_separable, pin3d_exact_small, pin3d_shift_axis2,
           pin3d_parseval_ortho, pin3d_adjoint_matrix, pin3d_adjoint_dot_fd]

ALL_PINS = [pin_matrix_form, pin_fft2, pin_mixed_radix, pin_whole_array, pin_exact_small, pin_impulse,
            pin_constant, pin_onbin_exponential, pin_onbin_cosine, pin_parseval,
            pin_shift_theorem, pin_linearity_and_sampling, pin_adjoint_dot,
            pin_adjoint_sampled, pin_quadratic_fd] + PINS_3D
