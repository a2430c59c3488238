"""Parity of the per-window FFT comparator (the 2D SWFFT of Table 1 and
Fig. 4) against the FP64 oracle, through the C ABI, and its agreement with
the tree (Sec. 4.6: both compute the same intermediate values).

Tolerance: normwise relative max error <= 1e-5, as for the tree."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def swd():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1707_08213_amd as swd
    return swd


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def run(swd, x_np, n0, n1, algo="swfft", norm="none"):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    if x.dim() == 2:
        x = x.unsqueeze(0)
    p = swd.Plan(x.shape[1], x.shape[2], n0, n1, dtype=x.dtype, batch=x.shape[0], norm=norm,
                 algo=algo)
    print(f"[case] {p.describe()}", flush=True)
    y = p.forward(x)
    torch.cuda.synchronize()
    return y.cpu().numpy(), p.describe()


SHAPES = [(n0, n1) for n0 in (1, 2, 4, 8, 16, 32) for n1 in (1, 2, 4, 8, 16, 32)]


@pytest.mark.parametrize("n0,n1", SHAPES, ids=lambda v: str(v))
def test_swfft_every_window_shape(swd, orc, n0, n1):
    """Several window groups and slabs, with a ragged last group."""
    wg = 64 // max(n0, n1)
    x = workloads.normal_real((2 * n0 + 21, 3 * wg + n1 + 2), seed=500 + n0 * 64 + n1)
    y, desc = run(swd, x, n0, n1)
    assert "algo=swfft" in desc
    ref = orc.swdft2d(x.astype(np.float64), n0, n1)
    assert y.shape[1:] == ref.shape
    assert rel_err(y[0], ref) <= TOL


@pytest.mark.parametrize("n0,n1", [(32, 8), (16, 16), (8, 32), (2, 4), (1, 32), (32, 1)],
                         ids=lambda v: str(v))
def test_swfft_complex_batch(swd, orc, n0, n1):
    N = (n0 + 17, 2 * (64 // max(n0, n1)) + n1 + 3)
    xs = np.stack([workloads.normal_complex(N, seed=600 + b + n0 + n1) for b in range(3)])
    y, _ = run(swd, xs, n0, n1)
    for b in range(3):
        assert rel_err(y[b], orc.swdft2d(xs[b].astype(np.complex128), n0, n1)) <= TOL, b


def test_swfft_ortho(swd, orc):
    x = workloads.normal_real((40, 50), seed=9)
    y, _ = run(swd, x, 8, 16, norm="ortho")
    assert rel_err(y[0], orc.swdft2d(x.astype(np.float64), 8, 16, norm="ortho")) <= TOL


def test_swfft_exact_gaussian_integers(swd):
    """n_i <= 4: every twiddle is a power of -i, so integer inputs give exact
    integer outputs."""
    rng = np.random.default_rng(11)
    x = (rng.integers(-9, 10, size=(23, 37)) + 1j * rng.integers(-9, 10, size=(23, 37)))
    x = x.astype(np.complex64)
    y, _ = run(swd, x, 4, 2)
    win = np.lib.stride_tricks.sliding_window_view(x.astype(np.complex128), (4, 2))
    assert np.array_equal(y[0], np.rint(np.fft.fft2(win, axes=(-2, -1))))


@pytest.mark.parametrize("n0,n1", [(16, 16), (4, 4), (2, 8), (32, 16), (16, 32)],
                         ids=lambda v: str(v))
def test_swfft_agrees_with_tree(swd, n0, n1):
    """Sec. 4.6: the tree and the per-window FFT perform the same butterflies
    on the same values, so they agree to a few FP32 rounding steps (not
    bitwise: the compiler may fuse a multiply and an add in one kernel and
    not in the other, and split streams fold twiddles)."""
    x = workloads.normal_real((n0 + 70, n1 + 90), seed=700 + n0 + n1)
    a, _ = run(swd, x, n0, n1, algo="swfft")
    t, _ = run(swd, x, n0, n1, algo="tree")
    assert rel_err(a, t) <= 2e-6


def test_sin1024_swfft_sampled(swd, orc):
    """The 1024x1024 / 16x16 workload through the comparator: 4096 sampled
    windows (corners and edges included) against the oracle."""
    w = workloads.sin1024()
    x = torch.from_numpy(w["x"]).cuda()
    print("[case] sin1024 swfft full size", flush=True)
    y = swd.swdft2d(x, 16, 16, algo="swfft")
    q0, q1 = workloads.window_sample(1009, 1009, 4096, 2001)
    got = y[torch.from_numpy(q0).cuda(), torch.from_numpy(q1).cuda()].cpu().numpy()
    del y
    torch.cuda.empty_cache()
    ref = orc.swdft2d(w["x"].astype(np.float64), 16, 16, windows=(q0, q1))
    assert rel_err(got, ref) <= TOL
