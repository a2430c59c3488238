"""Parity of the mixed-radix tree (window sides 2^a 3^b, the radix-3 and
mixed trees of Sec. 5) and of the FP64 direct kernel on such windows, against
the FP64 oracle, through the C ABI.

Tolerance: normwise relative max error <= 1e-5 for the FP32 tree, <= 1e-12
for the FP64 direct kernel."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

TOL = 1e-5

ODD = (3, 6, 9, 12, 24)
SHAPES = ([(a, b) for a in ODD for b in ODD + (4, 8, 16)] +
          [(a, b) for a in (4, 8, 16) for b in ODD])


@pytest.fixture(scope="module")
def swd():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1707_08213_amd as swd
    return swd


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def describe_field(desc, key):
    return int(desc.split(f" {key}=")[1].split()[0])


def run(swd, x_np, n0, n1, algo="tree", norm="none"):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    if x.dim() == 2:
        x = x.unsqueeze(0)
    p = swd.Plan(x.shape[1], x.shape[2], n0, n1, dtype=x.dtype, batch=x.shape[0], norm=norm,
                 algo=algo)
    print(f"[case] {p.describe()}", flush=True)
    y = p.forward(x)
    torch.cuda.synchronize()
    return y.cpu().numpy(), p.describe()


@pytest.mark.parametrize("n0,n1", SHAPES, ids=lambda v: str(v))
def test_mixed_tree_every_shape(swd, orc, monkeypatch, n0, n1):
    """One-chunk slabs (priming rows at every slab top), several strips and a
    ragged last strip and slab."""
    desc = swd.Plan(400, 400, n0, n1).describe()
    cr = describe_field(desc, "rows_per_chunk")
    cols = describe_field(desc, "cols_per_wave")
    assert "radix=2,3" in desc
    monkeypatch.setenv("SWDFT_TREE_SLAB", str(cr))
    x = workloads.normal_real((n0 - 1 + 2 * cr + 7, n1 - 1 + 3 * cols + 2),
                              seed=1100 + 31 * n0 + n1)
    y, d = run(swd, x, n0, n1)
    assert describe_field(d, "slabs") == 3, d
    ref = orc.swdft2d(x.astype(np.float64), n0, n1)
    assert y.shape[1:] == ref.shape
    assert rel_err(y[0], ref) <= TOL


@pytest.mark.parametrize("n0,n1", [(12, 9), (24, 3), (6, 16), (9, 24)], ids=lambda v: str(v))
def test_mixed_tree_complex_batch(swd, orc, n0, n1):
    N = (n0 + 61, n1 + 2 * (64 // n1) + 3)
    xs = np.stack([workloads.normal_complex(N, seed=1200 + b + n0 + n1) for b in range(2)])
    y, _ = run(swd, xs, n0, n1)
    for b in range(2):
        assert rel_err(y[b], orc.swdft2d(xs[b].astype(np.complex128), n0, n1)) <= TOL, b


def test_mixed_tree_ortho(swd, orc):
    x = workloads.normal_real((50, 41), seed=13)
    y, _ = run(swd, x, 6, 12, norm="ortho")
    assert rel_err(y[0], orc.swdft2d(x.astype(np.float64), 6, 12, norm="ortho")) <= TOL


@pytest.mark.parametrize("n0,n1", [(12, 9), (3, 24), (24, 8)], ids=lambda v: str(v))
def test_direct_f64_mixed(swd, orc, n0, n1):
    """The FP64 direct kernel steps (j k) mod n for any n."""
    x = workloads.normal_complex((n0 + 9, n1 + 11), seed=1300 + n0 + n1).astype(np.complex128)
    y, _ = run(swd, x, n0, n1, algo="direct_f64")
    assert rel_err(y[0], orc.swdft2d(x, n0, n1)) <= 1e-12


@pytest.mark.parametrize("n", [12, 24])
def test_mixed_tree_1024_sampled(swd, orc, n):
    """1024 x 1024 real image (the headline size) with n x n windows of the
    mixed kernel, default launch: 512 sampled windows against the oracle."""
    x = workloads.normal_real((1024, 1024), seed=1400 + n)
    xt = torch.from_numpy(x).cuda()
    print(f"[case] 1024x1024 {n}x{n} mixed", flush=True)
    y = swd.swdft2d(xt, n, n)
    P = 1024 - n + 1
    q0, q1 = workloads.window_sample(P, P, 512, 1401)
    got = y[torch.from_numpy(q0).cuda(), torch.from_numpy(q1).cuda()].cpu().numpy()
    del y
    torch.cuda.empty_cache()
    ref = orc.swdft2d(x.astype(np.float64), n, n, windows=(q0, q1))
    assert rel_err(got, ref) <= TOL


def test_mixed_tree_tuned_and_capped(swd, orc, monkeypatch):
    """The tuner's pick (slab and resident cap; streams stay whole) and an
    explicit one-workgroup-per-CU cap both give the transform."""
    x = workloads.normal_real((300, 260), seed=1500)
    xt = torch.from_numpy(x).cuda().unsqueeze(0)
    q0, q1 = workloads.window_sample(300 - 12 + 1, 260 - 12 + 1, 256, 1501)
    ref = orc.swdft2d(x.astype(np.float64), 12, 12, windows=(q0, q1))
    p = swd.Plan(300, 260, 12, 12)
    p.tune(xt)
    print(f"[case] tuned {p.describe()}", flush=True)
    assert " kg=1 " in p.describe() and " waves_per_strip=1 " in p.describe()
    y = p.forward(xt)[0]
    got = y[torch.from_numpy(q0).cuda(), torch.from_numpy(q1).cuda()].cpu().numpy()
    assert rel_err(got, ref) <= TOL
    monkeypatch.setenv("SWDFT_TREE_WPC", "1")
    y1, d = run(swd, x, 12, 12)
    assert " groups_per_cu=1 " in d, d
    got1 = y1[0][q0, q1]
    assert rel_err(got1, ref) <= TOL
