"""Seeded synthetic inputs for the 2D sliding-window DFT workloads.

This module only draws random numbers and arranges them into arrays; it holds
no part of the transform's arithmetic. Both the FP64 oracle tests and the HIP
path's tests/bench draw their inputs from here, so the two sides see exactly
the same values.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) and draws in
FP64; FP32 inputs are rounded once from those draws.

Workloads (sizes follow the problem statement of the 2D SWDFT, Sec. 4.1:
an N0 x N1 array, n0 x n1 radix-2 windows, P_i = N_i - n_i + 1 positions):

* ``small64``  - 64x64 real FP64, N(0,1), 4x4 windows.
* ``sin1024``  - 1024x1024 real FP32, N(0,1) plus three planted on-bin 2D
  cosines of amplitude 5, 16x16 windows.
* ``cplx2048`` - 2048x512 complex64 (re, im i.i.d. N(0,1)), 32x8 windows.
* ``uneven64`` - 64 real FP32 images, each side drawn from {128,256,512,1024},
  window drawn from {8x8, 16x16, 32x32, 8x32}.
* ``grad256``  - batch of 16 real FP32 256x256 images, 16x16 windows, with a
  Bernoulli(0.25) frequency band mask for the loss sum w*|A|^2.
"""
from __future__ import annotations

import numpy as np

WORKLOAD_SEEDS = {"small64": 1, "sin1024": 2, "cplx2048": 3, "uneven64": 4, "grad256": 5,
                  "vol128": 6, "fig4": 7, "mixed1024": 8}

UNEVEN_SIDES = (128, 256, 512, 1024)
UNEVEN_WINDOWS = ((8, 8), (16, 16), (32, 32), (8, 32))


def rng_for(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def normal_real(shape, seed: int, dtype=np.float32) -> np.ndarray:
    """i.i.d. N(0,1) drawn in FP64, then rounded once to ``dtype``."""
    return rng_for(seed).standard_normal(shape).astype(dtype)


def normal_complex(shape, seed: int, dtype=np.complex64) -> np.ndarray:
    """Real and imaginary parts i.i.d. N(0,1) (real part drawn first)."""
    rng = rng_for(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im).astype(dtype)


def planted_cosines(N0: int, N1: int, n0: int, n1: int, count: int, amplitude: float,
                    rng: np.random.Generator):
    """Sum of ``count`` 2D cosines that are on-bin for every n0 x n1 window.

    Frequencies are f_i = k_i * N_i / n_i cycles per image with k_i drawn
    uniformly from [1, n_i/2) (distinct (k0,k1) pairs), so each window sees an
    integer number k_i of cycles. Phase is uniform on [0, 2*pi).
    Returns (array in FP64, list of (k0, k1, phase)).
    """
    lo0, hi0 = (1, max(2, n0 // 2))
    lo1, hi1 = (1, max(2, n1 // 2))
    picked = []
    while len(picked) < count:
        k0 = int(rng.integers(lo0, hi0))
        k1 = int(rng.integers(lo1, hi1))
        if (k0, k1) not in [(a, b) for a, b, _ in picked]:
            picked.append((k0, k1, float(rng.uniform(0.0, 2.0 * np.pi))))
    r = np.arange(N0, dtype=np.float64)[:, None]
    c = np.arange(N1, dtype=np.float64)[None, :]
    out = np.zeros((N0, N1), dtype=np.float64)
    for k0, k1, ph in picked:
        f0 = k0 * N0 // n0
        f1 = k1 * N1 // n1
        out += amplitude * np.cos(2.0 * np.pi * (f0 * r / N0 + f1 * c / N1) + ph)
    return out, picked


def window_sample(P0: int, P1: int, count: int, seed: int):
    """Seeded sample of window positions (q0, q1), always holding the four
    corners, the four edge midpoints and the centre. Returns two int64 arrays."""
    fixed = {(0, 0), (0, P1 - 1), (P0 - 1, 0), (P0 - 1, P1 - 1),
             (0, P1 // 2), (P0 - 1, P1 // 2), (P0 // 2, 0), (P0 // 2, P1 - 1),
             (P0 // 2, P1 // 2)}
    fixed = sorted(fixed)
    total = P0 * P1
    count = min(count, total)
    rng = rng_for(seed)
    chosen = {a * P1 + b for a, b in fixed}
    if count > len(chosen):
        extra = rng.choice(total, size=min(total, count + len(chosen)), replace=False)
        for e in extra:
            if len(chosen) >= count:
                break
            chosen.add(int(e))
    flat = np.array(sorted(chosen), dtype=np.int64)
    return flat // P1, flat % P1


def window_sample3(P, count: int, seed: int):
    """Seeded sample of 3D window positions (q0, q1, q2) in [0, P_i), always
    holding the eight corners and the centre. Returns three int64 arrays."""
    P0, P1, P2 = (int(v) for v in P)
    fixed = {(a, b, c) for a in (0, P0 - 1) for b in (0, P1 - 1) for c in (0, P2 - 1)}
    fixed.add((P0 // 2, P1 // 2, P2 // 2))
    total = P0 * P1 * P2
    count = min(count, total)
    chosen = {(a * P1 + b) * P2 + c for a, b, c in fixed}
    rng = rng_for(seed)
    if count > len(chosen):
        extra = rng.choice(total, size=min(total, count + len(chosen)), replace=False)
        for e in extra:
            if len(chosen) >= count:
                break
            chosen.add(int(e))
    flat = np.array(sorted(chosen), dtype=np.int64)
    return flat // (P1 * P2), (flat // P2) % P1, flat % P2


def pixel_sample(N0: int, N1: int, count: int, seed: int):
    """Seeded sample of input pixels (r, c), always holding corners and edges."""
    return window_sample(N0, N1, count, seed)


def band_mask(n0: int, n1: int, p: float, seed: int) -> np.ndarray:
    """w in {0,1}^{n0 x n1}, i.i.d. Bernoulli(p), as float32."""
    return (rng_for(seed).random((n0, n1)) < p).astype(np.float32)


# ---------------------------------------------------------------- workloads

def small64(seed: int = WORKLOAD_SEEDS["small64"]):
    return dict(x=normal_real((64, 64), seed, np.float64), n0=4, n1=4)


def sin1024(seed: int = WORKLOAD_SEEDS["sin1024"], N0: int = 1024, N1: int = 1024,
            n0: int = 16, n1: int = 16):
    rng = rng_for(seed)
    noise = rng.standard_normal((N0, N1))
    planted, freqs = planted_cosines(N0, N1, n0, n1, 3, 5.0, rng)
    return dict(x=(noise + planted).astype(np.float32), n0=n0, n1=n1, planted=freqs)


def mixed1024(seed: int = WORKLOAD_SEEDS["mixed1024"], N0: int = 1024, N1: int = 1024,
              n0: int = 12, n1: int = 12):
    """1024 x 1024 real N(0,1) image for the mixed-radix (2 and 3) tree."""
    return dict(x=normal_real((N0, N1), seed), n0=n0, n1=n1)


def cplx2048(seed: int = WORKLOAD_SEEDS["cplx2048"], N0: int = 2048, N1: int = 512,
             n0: int = 32, n1: int = 8):
    return dict(x=normal_complex((N0, N1), seed), n0=n0, n1=n1)


def uneven64(seed: int = WORKLOAD_SEEDS["uneven64"], count: int = 64,
             sides=UNEVEN_SIDES, windows=UNEVEN_WINDOWS):
    """List of dicts {x (float32 N0xN1), n0, n1}. Sizes and window shapes are
    drawn first (for all images), then the pixel values image by image."""
    rng = rng_for(seed)
    shapes = []
    for _ in range(count):
        N0 = int(sides[int(rng.integers(0, len(sides)))])
        N1 = int(sides[int(rng.integers(0, len(sides)))])
        n0, n1 = windows[int(rng.integers(0, len(windows)))]
        shapes.append((N0, N1, n0, n1))
    images = []
    for (N0, N1, n0, n1) in shapes:
        images.append(dict(x=rng.standard_normal((N0, N1)).astype(np.float32), n0=n0, n1=n1))
    return images


def vol128(seed: int = WORKLOAD_SEEDS["vol128"], N: int = 128, n: int = 8):
    """One N x N x N real FP32 volume, N(0,1), with n x n x n windows (the 3D
    extension of Sec. 4.4): 121^3 windows of 512 coefficients at the defaults."""
    return dict(x=normal_real((N, N, N), seed), n=(n, n, n))


def grad256(seed: int = WORKLOAD_SEEDS["grad256"], batch: int = 16, N: int = 256,
            n0: int = 16, n1: int = 16, p: float = 0.25):
    rng = rng_for(seed)
    x = rng.standard_normal((batch, N, N)).astype(np.float32)
    w = (rng.random((n0, n1)) < p).astype(np.float32)
    return dict(x=x, n0=n0, n1=n1, w=w)
