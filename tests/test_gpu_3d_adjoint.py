"""Parity of the 3D adjoint (the transposed tree of the k-dimensional
extension of Sec. 4.4, k = 3) through the C ABI and autograd, against the
oracle's explicit 3D adjoint, the dot-product identity and exact central
differences of a quadratic loss."""
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


SHAPES = [(n0, n1, n2) for n0 in (2, 4, 8, 16) for n1 in (2, 4, 8) for n2 in (2, 4, 8)]


@pytest.mark.parametrize("n0,n1,n2", SHAPES, ids=lambda v: str(v))
def test_adjoint3d_every_window_shape(swd, orc, n0, n1, n2):
    """Every supported window shape, real and complex dx, volumes that leave
    ragged strips along axis 2 and more than one slab along axis 0."""
    qw = 64 // (n1 * n2)
    N = (2 * n0 + 5, n1 + 3, 2 * qw + n2 + 3)
    P = tuple(N[i] - (n0, n1, n2)[i] + 1 for i in range(3))
    rng = np.random.default_rng(500 + 64 * n0 + 8 * n1 + n2)
    dy = (rng.standard_normal(P + (n0, n1, n2)) +
          1j * rng.standard_normal(P + (n0, n1, n2))).astype(np.complex64)
    ref = orc.swdft3d_adjoint(dy.astype(np.complex128), *N)
    d = torch.from_numpy(dy).cuda()
    print(f"[case] 3D backward N={N} n={(n0, n1, n2)}", flush=True)
    got = swd.swdft3d_backward(d, *N, dtype=torch.float32).cpu().numpy()
    assert got.shape == N
    assert rel_err(got, ref.real) <= TOL
    gotc = swd.swdft3d_backward(d, *N, dtype=torch.complex64).cpu().numpy()
    assert rel_err(gotc, ref) <= TOL


@pytest.mark.parametrize("slab", [4, 8, 16])
def test_adjoint3d_slabs_and_batch(swd, orc, monkeypatch, slab):
    """Several slabs along axis 0 (each primed by the n0 - 1 window rows
    below it), a batch of two volumes, and the orthonormal scale."""
    monkeypatch.setenv("SWDFT3D_ADJ_SLAB", str(slab))
    n = (8, 4, 4)
    N = (37, 9, 14)
    P = tuple(N[i] - n[i] + 1 for i in range(3))
    rng = np.random.default_rng(77 + slab)
    dy = (rng.standard_normal((2,) + P + n) + 1j * rng.standard_normal((2,) + P + n)).astype(np.complex64)
    plan = swd.Plan3D(*N, *n, dtype=torch.complex64, batch=2, norm="ortho")
    got = plan.backward(torch.from_numpy(dy).cuda()).cpu().numpy()
    for b in range(2):
        ref = orc.swdft3d_adjoint(dy[b].astype(np.complex128), *N, norm="ortho")
        assert rel_err(got[b], ref) <= TOL


def test_adjoint3d_dot_product(swd):
    """<M x, g> = <x, M^H g> with both sides on the GPU."""
    rng = np.random.default_rng(41)
    N, n = (20, 11, 13), (4, 2, 8)
    P = tuple(N[i] - n[i] + 1 for i in range(3))
    x = rng.standard_normal(N).astype(np.float32)
    g = (rng.standard_normal(P + n) + 1j * rng.standard_normal(P + n)).astype(np.complex64)
    mx = swd.swdft3d(torch.from_numpy(x).cuda(), *n).cpu().numpy().astype(np.complex128)
    mhg = swd.swdft3d_backward(torch.from_numpy(g).cuda(), *N).cpu().numpy().astype(np.float64)
    lhs = np.real(np.vdot(g.astype(np.complex128), mx))
    rhs = np.sum(x.astype(np.float64) * mhg)
    assert abs(lhs - rhs) <= 1e-5 * np.sqrt(np.sum(np.abs(g) ** 2) * np.sum(np.abs(mx) ** 2))


def test_autograd3d_quadratic_loss_fd(swd, orc):
    """L = sum w |A|^2 with a Bernoulli(0.3) mask over (k0, k1, k2): x.grad
    through SWDFT3dFn against the oracle adjoint of 2 w A and exact FP64
    central differences (h = 1) of L at corner and interior voxels."""
    rng = np.random.default_rng(43)
    N, n = (14, 10, 12), (4, 4, 2)
    x_np = rng.standard_normal(N).astype(np.float32)
    w_np = (rng.random(n) < 0.3).astype(np.float32)
    w_np[1, 0, 1] = 1.0
    x = torch.from_numpy(x_np).cuda().requires_grad_(True)
    w = torch.from_numpy(w_np).cuda()
    A = swd.SWDFT3dFn.apply(x, *n)
    (w * A.abs() ** 2).sum().backward()
    grad = x.grad.cpu().numpy().astype(np.float64)
    xd = x_np.astype(np.float64)
    A_ref = orc.swdft3d(xd, *n)
    grad_ref = orc.swdft3d_adjoint(2.0 * w_np * A_ref, *N).real
    assert rel_err(grad, grad_ref) <= TOL

    def L(z):
        return float(np.sum(w_np * np.abs(orc.swdft3d(z, *n)) ** 2))

    for v in [(0, 0, 0), (13, 9, 11), (5, 4, 6), (0, 9, 0), (13, 0, 11)]:
        e = np.zeros_like(xd)
        e[v] = 1.0
        fd = (L(xd + e) - L(xd - e)) / 2.0
        assert abs(grad[v] - fd) <= TOL * np.max(np.abs(grad_ref)), v


def test_adjoint3d_vol128_boxes(swd, orc):
    """128^3 real FP32, 8 x 8 x 8 windows (the vol128 workload's shape): the
    adjoint of a random dy on three 4^3 voxel boxes (both corners of the
    volume and its centre). The oracle gets the windows that cover a box (a
    sub-volume's worth of dy), which is all that its voxels depend on."""
    n = (8, 8, 8)
    N = (128, 128, 128)
    P = tuple(N[i] - n[i] + 1 for i in range(3))
    g = torch.Generator(device="cuda").manual_seed(9)
    dy = torch.complex(torch.randn(P + n, device="cuda", generator=g),
                       torch.randn(P + n, device="cuda", generator=g))
    print("[case] 3D backward vol128", flush=True)
    dx = swd.swdft3d_backward(dy, *N)
    for lo in [(0, 0, 0), (62, 62, 62), (124, 124, 124)]:
        hi = tuple(l + 4 for l in lo)
        xl = tuple(max(0, lo[i] - n[i] + 1) for i in range(3))
        xh = tuple(min(N[i], hi[i] + n[i] - 1) for i in range(3))
        sub = tuple(slice(xl[i], xh[i] - n[i] + 1) for i in range(3))
        dys = dy[sub].cpu().numpy().astype(np.complex128)
        ref = orc.swdft3d_adjoint(dys, *(xh[i] - xl[i] for i in range(3)))
        ref = ref[tuple(slice(lo[i] - xl[i], hi[i] - xl[i]) for i in range(3))]
        got = dx[tuple(slice(lo[i], hi[i]) for i in range(3))].cpu().numpy()
        assert rel_err(got, ref.real) <= TOL, lo
