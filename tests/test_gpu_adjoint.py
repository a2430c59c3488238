"""The hand-written adjoint (transposed tree) through the C ABI and autograd,
against the oracle's explicit adjoint, the dot-product identity and exact
central differences of a quadratic loss."""
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


def gpu_backward(swd, dy_np, N0, N1, dtype, norm="none"):
    dy = torch.from_numpy(np.ascontiguousarray(dy_np)).cuda()
    print(f"[case] backward N={N0}x{N1} n={dy_np.shape[-2]}x{dy_np.shape[-1]} {dtype}", flush=True)
    dx = swd.swdft2d_backward(dy, N0, N1, dtype=dtype, norm=norm)
    torch.cuda.synchronize()
    return dx.cpu().numpy()


SHAPES = [(n0, n1) for n0 in (1, 2, 4, 8, 16, 32) for n1 in (1, 2, 4, 8, 16, 32)]


@pytest.mark.parametrize("n0,n1", SHAPES, ids=lambda v: str(v))
def test_adjoint_every_window_shape(swd, orc, n0, n1):
    N0 = 2 * n0 + 21
    N1 = 2 * (64 // n1) + n1 + 3
    P0, P1 = N0 - n0 + 1, N1 - n1 + 1
    rng = np.random.default_rng(1000 + 64 * n0 + n1)
    dy = (rng.standard_normal((P0, P1, n0, n1)) + 1j * rng.standard_normal((P0, P1, n0, n1)))
    dy = dy.astype(np.complex64)
    got = gpu_backward(swd, dy, N0, N1, torch.float32)
    ref = orc.swdft2d_adjoint(dy.astype(np.complex128), N0, N1).real
    assert got.shape == (N0, N1)
    assert rel_err(got, ref) <= TOL
    gotc = gpu_backward(swd, dy, N0, N1, torch.complex64)
    refc = orc.swdft2d_adjoint(dy.astype(np.complex128), N0, N1)
    assert rel_err(gotc, refc) <= TOL


@pytest.mark.parametrize("n0,n1,slab", [(16, 16, 16), (32, 8, 32), (8, 4, 8), (4, 32, 32),
                                        (2, 2, 2)])
def test_adjoint_slab_boundaries(swd, orc, n0, n1, slab):
    """Several row slabs per image (each primed by the n0-1 window rows below
    it) and several strips: the priming and the workspace reduction must
    reproduce the single-slab result."""
    N0, N1 = 5 * slab + n0 + 3, 3 * (64 // n1) + n1 + 7
    P0, P1 = N0 - n0 + 1, N1 - n1 + 1
    rng = np.random.default_rng(7)
    dy = (rng.standard_normal((2, P0, P1, n0, n1)) +
          1j * rng.standard_normal((2, P0, P1, n0, n1))).astype(np.complex64)
    os.environ["SWDFT_ADJ_SLAB"] = str(slab)
    try:
        got = gpu_backward(swd, dy, N0, N1, torch.float32)
    finally:
        del os.environ["SWDFT_ADJ_SLAB"]
    for b in range(2):
        ref = orc.swdft2d_adjoint(dy[b].astype(np.complex128), N0, N1).real
        assert rel_err(got[b], ref) <= TOL


@pytest.mark.parametrize("kg", [1, 2])
@pytest.mark.parametrize("n0,n1,slab", [(8, 1, 0), (8, 8, 16), (16, 4, 0), (16, 16, 32),
                                        (16, 32, 0), (32, 1, 0), (32, 8, 16), (32, 16, 32),
                                        (32, 32, 0)])
def test_adjoint_lane_split(swd, orc, monkeypatch, n0, n1, slab, kg):
    """A column stream of the adjoint split over one or two lanes by k0
    residue (two lanes exchange their level-1 nodes), real and complex, with
    one slab or several (slab > 0): both against the oracle's explicit
    adjoint (the transpose of Eq. (5)-(6))."""
    monkeypatch.setenv("SWDFT_ADJ_KG", str(kg))
    if slab:
        monkeypatch.setenv("SWDFT_ADJ_SLAB", str(slab))
    N0 = (3 * slab if slab else 2 * n0) + n0 + 5
    N1 = 3 * (64 // (n1 * kg)) + n1 + 5
    P0, P1 = N0 - n0 + 1, N1 - n1 + 1
    rng = np.random.default_rng(31 + 64 * n0 + n1 + kg)
    dy = (rng.standard_normal((P0, P1, n0, n1)) +
          1j * rng.standard_normal((P0, P1, n0, n1))).astype(np.complex64)
    got = gpu_backward(swd, dy, N0, N1, torch.float32)
    ref = orc.swdft2d_adjoint(dy.astype(np.complex128), N0, N1)
    assert rel_err(got, ref.real) <= TOL
    gotc = gpu_backward(swd, dy, N0, N1, torch.complex64)
    assert rel_err(gotc, ref) <= TOL


@pytest.mark.parametrize("n0,n1,slab", [(16, 16, 16), (32, 8, 32), (4, 2, 4), (8, 32, 32)])
def test_forward_slab_boundaries(swd, orc, n0, n1, slab):
    """Forward with many slabs: the n0-1 priming rows at each slab top."""
    N0, N1 = 4 * slab + n0 + 5, 2 * (64 // n1) + n1 + 3
    x = workloads.normal_real((N0, N1), seed=n0 + n1 + slab)
    os.environ["SWDFT_TREE_SLAB"] = str(slab)
    try:
        y = swd.swdft2d(torch.from_numpy(x).cuda(), n0, n1).cpu().numpy()
    finally:
        del os.environ["SWDFT_TREE_SLAB"]
    assert rel_err(y, orc.swdft2d(x.astype(np.float64), n0, n1)) <= TOL


def test_adjoint_dot_product(swd):
    """<M x, g> = <x, M^H g> with both sides on the GPU."""
    rng = np.random.default_rng(3)
    N0, N1, n0, n1 = 90, 70, 16, 8
    x = rng.standard_normal((N0, N1)).astype(np.float32)
    g = (rng.standard_normal((N0 - n0 + 1, N1 - n1 + 1, n0, n1)) +
         1j * rng.standard_normal((N0 - n0 + 1, N1 - n1 + 1, n0, n1))).astype(np.complex64)
    mx = swd.swdft2d(torch.from_numpy(x).cuda(), n0, n1).cpu().numpy().astype(np.complex128)
    mhg = gpu_backward(swd, g, N0, N1, torch.float32).astype(np.float64)
    lhs = np.real(np.vdot(g.astype(np.complex128), mx))
    rhs = np.sum(x.astype(np.float64) * mhg)
    assert abs(lhs - rhs) <= 1e-5 * np.sqrt(np.sum(np.abs(g) ** 2) * np.sum(np.abs(mx) ** 2))


def test_adjoint_ortho(swd, orc):
    rng = np.random.default_rng(4)
    N0, N1, n0, n1 = 40, 50, 8, 8
    dy = (rng.standard_normal((N0 - 7, N1 - 7, 8, 8)) + 0j).astype(np.complex64)
    got = gpu_backward(swd, dy, N0, N1, torch.float32, norm="ortho")
    ref = orc.swdft2d_adjoint(dy.astype(np.complex128), N0, N1, norm="ortho").real
    assert rel_err(got, ref) <= TOL


def test_autograd_quadratic_loss_fd(swd, orc):
    """L = sum w |A|^2 with a Bernoulli(0.25) band mask: x.grad from autograd
    (which calls the adjoint kernel) against the oracle adjoint of 2 w A and
    against exact FP64 central differences of L."""
    rng = np.random.default_rng(6)
    N0, N1, n0, n1 = 36, 44, 8, 16
    x_np = rng.standard_normal((N0, N1)).astype(np.float32)
    w_np = workloads.band_mask(n0, n1, 0.25, 9)
    x = torch.from_numpy(x_np).cuda().requires_grad_(True)
    w = torch.from_numpy(w_np).cuda()
    A = swd.SWDFT2dFn.apply(x, n0, n1)
    loss = (w * A.abs() ** 2).sum()
    loss.backward()
    grad = x.grad.cpu().numpy().astype(np.float64)
    xd = x_np.astype(np.float64)
    A_ref = orc.swdft2d(xd, n0, n1)
    grad_ref = orc.swdft2d_adjoint(2.0 * w_np * A_ref, N0, N1).real
    assert rel_err(grad, grad_ref) <= TOL

    def L(z):
        return float(np.sum(w_np * np.abs(orc.swdft2d(z, n0, n1)) ** 2))

    for (r, c) in [(0, 0), (N0 - 1, N1 - 1), (17, 23), (0, N1 - 1), (N0 - 1, 0), (9, 40)]:
        e = np.zeros_like(xd)
        e[r, c] = 1.0
        fd = (L(xd + e) - L(xd - e)) / 2.0
        assert abs(grad[r, c] - fd) <= TOL * np.max(np.abs(grad_ref)), (r, c)


def test_autograd_gradcheck_small(swd):
    """torch.autograd.gradcheck-style check in FP32 on a tiny complex input
    (complex x: the adjoint returns the full complex M^H dy)."""
    rng = np.random.default_rng(8)
    N0, N1, n0, n1 = 9, 12, 4, 4
    x = torch.from_numpy((rng.standard_normal((N0, N1)) +
                          1j * rng.standard_normal((N0, N1))).astype(np.complex64)).cuda()
    x.requires_grad_(True)
    g = torch.from_numpy((rng.standard_normal((N0 - 3, N1 - 3, 4, 4)) +
                          1j * rng.standard_normal((N0 - 3, N1 - 3, 4, 4))).astype(np.complex64)).cuda()
    A = swd.SWDFT2dFn.apply(x, n0, n1)
    (A * g.conj()).real.sum().backward()
    # d/dx Re<g, A> with PyTorch's conjugate-Wirtinger convention is M^H g
    ref = swd.swdft2d_backward(g, N0, N1, dtype=torch.complex64)
    assert torch.allclose(x.grad, ref, rtol=1e-5, atol=1e-5)


def test_grad256_sampled(swd, orc):
    """16 x 256 x 256 real FP32, 16 x 16 windows, L = sum w |A|^2 with a
    Bernoulli(0.25) band mask: gradient on 256 sampled pixels (corners and
    edges included) of two images against the oracle adjoint applied to the
    same dy = 2 w A."""
    wl = workloads.grad256()
    x = torch.from_numpy(wl["x"]).cuda().requires_grad_(True)
    w = torch.from_numpy(wl["w"]).cuda()
    print("[case] grad256 forward+backward", flush=True)
    A = swd.SWDFT2dFn.apply(x, 16, 16)
    dy = (2.0 * w * A).detach()
    (w * A.abs() ** 2).sum().backward()
    torch.cuda.synchronize()
    r, c = workloads.pixel_sample(256, 256, 256, 55)
    for b in (0, 15):
        dy_b = dy[b].cpu().numpy().astype(np.complex128)
        ref = orc.swdft2d_adjoint(dy_b, 256, 256, pixels=(r, c)).real
        got = x.grad[b].cpu().numpy()[r, c]
        assert rel_err(got, ref) <= TOL, b


def test_backward_rejects_direct_plan(swd):
    p = swd.Plan(32, 32, 4, 4, dtype=torch.float64, algo="direct_f64")
    dy = torch.zeros(p.out_shape, dtype=torch.complex128, device="cuda")
    with pytest.raises(swd.SwdftError) as e:
        p.backward(dy)
    assert e.value.name == "SWDFT_E_DTYPE"


def test_backward_after_dense_tuning(swd, orc, tmp_path, monkeypatch):
    """A tuning-cache line that picks the dense variant for the forward pass
    of an AUTO plan must leave the adjoint (always the transposed tree)
    usable: forward through the dense kernel, then autograd's backward, both
    against the oracle (forward: the dense tolerance; gradient: the oracle's
    explicit adjoint of the same dy)."""
    N0, N1, n0, n1 = 41, 53, 16, 16
    P0, P1 = N0 - n0 + 1, N1 - n1 + 1
    size = int(P0 * P1).bit_length() - 1
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cache = tmp_path / "tune.jsonl"
    cache.write_text('{"arch":"%s","kind":"single","n0":%d,"n1":%d,"real":1,"size":%d,'
                     '"algo":"dense","kg":1,"slab":0,"wpc":-1,"wv":0,"us":1.0}\n'
                     % (arch, n0, n1, size))
    monkeypatch.setenv("SWDFT_AUTOTUNE_CACHE", str(cache))
    rng = np.random.default_rng(21)
    x_np = rng.standard_normal((N0, N1)).astype(np.float32)
    x = torch.from_numpy(x_np).cuda().requires_grad_(True)
    print("[case] forward (dense from the tuning cache) then backward", flush=True)
    A = swd.SWDFT2dFn.apply(x, n0, n1)
    g_np = (rng.standard_normal((P0, P1, n0, n1)) +
            1j * rng.standard_normal((P0, P1, n0, n1))).astype(np.complex64)
    g = torch.from_numpy(g_np).cuda()
    (A * g.conj()).real.sum().backward()
    torch.cuda.synchronize()
    plan = swd._cached_plan(N0, N1, n0, n1, torch.float32, 1, "none", "auto")
    assert "dense" in plan.describe(), plan.describe()
    A_ref = orc.swdft2d(x_np.astype(np.float64), n0, n1)
    assert rel_err(A.detach().cpu().numpy(), A_ref) <= 5e-5
    grad_ref = orc.swdft2d_adjoint(g_np.astype(np.complex128), N0, N1).real
    assert rel_err(x.grad.cpu().numpy(), grad_ref) <= TOL
