"""Parity of the 3D tree (the k-dimensional extension of Sec. 4.4, k = 3)
against the FP64 oracle, through the C ABI.

Tolerance: normwise relative max error <= 1e-5 (as for the 2D tree; the
measured error is ~2e-7)."""
import os

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


def gpu3(swd, x_np, n, norm="none", env=None):
    saved = {}
    for k, v in (env or {}).items():
        saved[k] = os.environ.get(k)
        os.environ[k] = str(v)
    try:
        xb = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
        if xb.dim() == 3:
            xb = xb.unsqueeze(0)
        p = swd.Plan3D(*xb.shape[1:], *n, dtype=xb.dtype, batch=xb.shape[0], norm=norm)
        print(f"[case] {p.describe()}", flush=True)
        y = p.forward(xb)
        torch.cuda.synchronize()
        return y.cpu().numpy(), p.describe()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


SHAPES = [(n0, n1, n2) for n0 in (2, 4, 8, 16) for n1 in (2, 4, 8) for n2 in (2, 4, 8)]


@pytest.mark.parametrize("n", SHAPES, ids=lambda v: "x".join(map(str, v)))
def test_tree3d_every_window_shape(swd, orc, n):
    """Several strips (64/(n1 n2) windows each), slabs and chunks, with ragged
    ends along every axis."""
    n0, n1, n2 = n
    qw = 64 // (n1 * n2)
    N = (n0 + 11, n1 + 3, 2 * qw + n2 + 3)
    x = workloads.normal_real(N, seed=300 + n0 * 100 + n1 * 10 + n2)
    y, _ = gpu3(swd, x, n)
    ref = orc.swdft3d(x.astype(np.float64), *n)
    assert y.shape[1:] == ref.shape
    assert rel_err(y[0], ref) <= TOL


@pytest.mark.parametrize("n", [(2, 2, 8), (8, 4, 2), (16, 8, 8), (4, 8, 4)],
                         ids=lambda v: "x".join(map(str, v)))
def test_tree3d_complex_batch(swd, orc, n):
    N = (n[0] + 6, n[1] + 2, 64 // (n[1] * n[2]) + n[2] + 5)
    xs = np.stack([workloads.normal_complex(N, seed=400 + b) for b in range(2)])
    y, _ = gpu3(swd, xs, n)
    for b in range(2):
        assert rel_err(y[b], orc.swdft3d(xs[b].astype(np.complex128), *n)) <= TOL, b


def test_tree3d_ortho_scale(swd, orc):
    x = workloads.normal_real((20, 12, 14), seed=5)
    n = (4, 8, 2)
    y, _ = gpu3(swd, x, n, norm="ortho")
    assert rel_err(y[0], orc.swdft3d(x.astype(np.float64), *n, norm="ortho")) <= TOL
    y1, _ = gpu3(swd, x, n)
    assert np.allclose(y1[0] / np.sqrt(64.0), y[0], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("env", [{"SWDFT3D_SLAB": 8}, {"SWDFT3D_WPC": 1, "SWDFT3D_SLAB": 8},
                                 {"SWDFT3D_WPC": 2}],
                         ids=["slab8", "cap1-slab8", "cap2"])
def test_tree3d_launch_shapes(swd, orc, env):
    """Short slabs (priming rows at every slab top), one or two resident
    workgroups per CU and dispatch-order rounds give the same transform."""
    x = workloads.normal_real((40, 30, 40), seed=6)
    n = (8, 4, 4)
    y, desc = gpu3(swd, x, n, env=env)
    if "SWDFT3D_WPC" in env:
        assert f"groups_per_cu={env['SWDFT3D_WPC']}" in desc, desc
    assert rel_err(y[0], orc.swdft3d(x.astype(np.float64), *n)) <= TOL


def test_tree3d_exact_gaussian_integers(swd):
    """n_i <= 4: every twiddle is a power of -i, so integer inputs give
    integer outputs; FP32 represents them exactly at these magnitudes."""
    rng = np.random.default_rng(7)
    x = (rng.integers(-8, 9, size=(9, 7, 10)) + 1j * rng.integers(-8, 9, size=(9, 7, 10)))
    x = x.astype(np.complex64)
    n = (4, 2, 4)
    y, _ = gpu3(swd, x, n)
    win = np.lib.stride_tricks.sliding_window_view(x.astype(np.complex128), n)
    ref = np.rint(np.fft.fftn(win, axes=(-3, -2, -1)))
    assert np.array_equal(y[0], ref)


def test_vol128_sampled(swd, orc):
    """128^3 real FP32 volume with 8x8x8 windows (121^3 windows, 7.26 GB of
    output): 256 sampled windows, corners and edges included, against the
    oracle."""
    w = workloads.vol128()
    x = torch.from_numpy(w["x"]).cuda()
    print("[case] vol128 full size", flush=True)
    y = swd.swdft3d(x, *w["n"])
    P = [x.shape[i] - w["n"][i] + 1 for i in range(3)]
    q = workloads.window_sample3(P, 256, 3001)
    got = y[tuple(torch.from_numpy(a).cuda() for a in q)].cpu().numpy()
    del y
    torch.cuda.empty_cache()
    ref = orc.swdft3d(w["x"].astype(np.float64), *w["n"], windows=q)
    assert rel_err(got, ref) <= TOL
