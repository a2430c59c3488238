"""Dense per-window variant (F_n0 X F_n1^T on the matrix cores, BF16 hi/lo
split products, FP32 accumulation) against the FP64 oracle.

Tolerance: each product a*b is formed as a_hi b_hi + a_hi b_lo + a_lo b_hi;
the dropped terms are below 3 * 2^-18 |a b| (about 1.1e-5 relative per
product), and two products are chained (row DFT, then column DFT), so the
normwise relative error stays below 5e-5 for well-scaled data. The measured
values (printed) are ~5e-6.
"""
import os

import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

TOL_DENSE = 5e-5


@pytest.fixture(scope="module")
def swd():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1707_08213_amd as swd
    return swd


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def dense(swd, x_np, n0, n1, norm="none"):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    print(f"[case] dense N={x_np.shape} n={n0}x{n1} {x_np.dtype}", flush=True)
    y = swd.swdft2d(x, n0, n1, norm=norm, algo="dense_bf16x2")
    torch.cuda.synchronize()
    return y.cpu().numpy()


SHAPES = [(a, b) for a in (8, 16, 32) for b in (8, 16, 32)]


@pytest.mark.parametrize("cplx", [False, True], ids=["real", "complex"])
@pytest.mark.parametrize("n0,n1", SHAPES, ids=lambda v: str(v))
def test_dense_every_shape(swd, orc, n0, n1, cplx):
    N0 = 2 * n0 + 53                       # several 16-row chunks, ragged
    N1 = 3 * max(1, 16 // n1) + n1 + 4     # several strips, ragged
    shape = (N0, N1)
    seed = 500 + 3 * n0 + n1 + int(cplx)
    x = workloads.normal_complex(shape, seed) if cplx else workloads.normal_real(shape, seed)
    y = dense(swd, x, n0, n1)
    ref = orc.swdft2d(x.astype(np.complex128 if cplx else np.float64), n0, n1)
    err = rel_err(y, ref)
    print(f"dense {n0}x{n1} {'complex' if cplx else 'real'}: normwise rel err {err:.2e}")
    assert err <= TOL_DENSE


@pytest.mark.parametrize("n0,n1,slab", [(32, 8, 16), (16, 16, 32), (8, 32, 16)])
def test_dense_slab_boundaries(swd, orc, n0, n1, slab):
    """Many slabs: each recomputes the row products of the n0 - 1 rows above."""
    N0, N1 = 6 * slab + n0 + 9, 2 * max(1, 16 // n1) + n1 + 3
    x = workloads.normal_complex((N0, N1), seed=n0 + n1 + slab)
    os.environ["SWDFT_DENSE_SLAB"] = str(slab)
    try:
        y = dense(swd, x, n0, n1)
    finally:
        del os.environ["SWDFT_DENSE_SLAB"]
    assert rel_err(y, orc.swdft2d(x.astype(np.complex128), n0, n1)) <= TOL_DENSE


def test_dense_ortho_and_batch(swd, orc):
    x = workloads.normal_real((3, 60, 70), seed=12)
    xt = torch.from_numpy(x).cuda()
    y = swd.swdft2d(xt, 16, 8, norm="ortho", algo="dense_bf16x2").cpu().numpy()
    for b in range(3):
        ref = orc.swdft2d(x[b].astype(np.float64), 16, 8, norm="ortho")
        assert rel_err(y[b], ref) <= TOL_DENSE


def test_dense_agrees_with_tree(swd):
    x = torch.from_numpy(workloads.normal_real((200, 150), seed=13)).cuda()
    a = swd.swdft2d(x, 16, 16, algo="dense_bf16x2")
    t = swd.swdft2d(x, 16, 16, algo="tree")
    err = float((a - t).abs().max() / t.abs().max())
    assert err <= TOL_DENSE


def test_dense_cplx2048_sampled(swd, orc):
    """2048 x 512 complex64, 32 x 8 windows: 4096 sampled windows; the error
    of the BF16 hi/lo products is reported."""
    w = workloads.cplx2048()
    x = torch.from_numpy(w["x"]).cuda()
    y = swd.swdft2d(x, 32, 8, algo="dense_bf16x2")
    P0, P1 = 2048 - 31, 512 - 7
    q0, q1 = workloads.window_sample(P0, P1, 4096, 1003)
    got = y[torch.from_numpy(q0).cuda(), torch.from_numpy(q1).cuda()].cpu().numpy()
    del y
    ref = orc.swdft2d(w["x"].astype(np.complex128), 32, 8, windows=(q0, q1))
    err = rel_err(got, ref)
    per_win = np.max(np.abs(got - ref), axis=(1, 2)) / np.max(np.abs(ref), axis=(1, 2))
    print(f"cplx2048 dense: normwise {err:.2e}, worst window {per_win.max():.2e}, "
          f"max abs {np.max(np.abs(got - ref)):.2e}")
    assert err <= TOL_DENSE


def test_dense_rejects_unsupported_window(swd):
    with pytest.raises(swd.SwdftError) as e:
        swd.Plan(64, 64, 4, 8, algo="dense_bf16x2")
    assert e.value.name == "SWDFT_E_WINDOW"
    with pytest.raises(swd.SwdftError) as e:
        swd.Plan(64, 64, 8, 8, dtype=torch.float64, algo="dense_bf16x2")
    assert e.value.name == "SWDFT_E_DTYPE"
