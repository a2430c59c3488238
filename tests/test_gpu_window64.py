"""Windows of 64 (the largest of the Fig. 4 sweep) through the tree, the
per-window FFT and the FP64 direct kernel, against the FP64 oracle.

At n0 = n1 = 64 a window costs the oracle 4096 multiply-adds per coefficient,
so outputs are compared on a seeded sample of windows that always holds the
four corners and the edge midpoints (plus whole output rows at a slab seam);
the images still span several strips, slabs and chunks with ragged tails.

Tolerance: normwise relative max error <= 1e-5 (FP32 paths), <= 1e-12 (FP64).
"""
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


def run_sampled(swd, orc, x_np, n0, n1, algo, count=96, seed=0, extra_rows=()):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda().unsqueeze(0)
    p = swd.Plan(x.shape[1], x.shape[2], n0, n1, dtype=x.dtype, algo=algo)
    print(f"[case] {p.describe()}", flush=True)
    y = p.forward(x)[0]
    torch.cuda.synchronize()
    P0, P1 = x_np.shape[0] - n0 + 1, x_np.shape[1] - n1 + 1
    q0, q1 = workloads.window_sample(P0, P1, count, seed)
    for r in extra_rows:
        q0 = np.concatenate([q0, np.full(P1, r, dtype=q0.dtype)])
        q1 = np.concatenate([q1, np.arange(P1, dtype=q1.dtype)])
    got = y[torch.from_numpy(q0).cuda(), torch.from_numpy(q1).cuda()].cpu().numpy()
    wide = np.float64 if x_np.dtype == np.float32 else np.complex128
    ref = orc.swdft2d(x_np.astype(wide), n0, n1, windows=(q0, q1))
    return got, ref, p.describe()


SHAPES64 = [(64, n1) for n1 in (1, 2, 4, 8, 16, 32, 64)] + [(n0, 64) for n0 in (1, 2, 4, 8, 16, 32)]


@pytest.mark.parametrize("n0,n1", SHAPES64, ids=lambda v: str(v))
def test_tree_window64_real(swd, orc, monkeypatch, n0, n1):
    """Short slabs (one chunk each) so that the image holds several slabs with
    priming rows; a ragged last strip and slab."""
    desc = swd.Plan(400, 400, n0, n1).describe()
    cr = int(desc.split("rows_per_chunk=")[1].split()[0])
    cols = int(desc.split("cols_per_wave=")[1].split()[0])
    monkeypatch.setenv("SWDFT_TREE_SLAB", str(cr))
    N0 = n0 - 1 + 2 * cr + 7
    N1 = n1 - 1 + 3 * cols + 2
    x = workloads.normal_real((N0, N1), seed=800 + n0 + 3 * n1)
    got, ref, d = run_sampled(swd, orc, x, n0, n1, "tree", seed=801 + n0 + n1,
                              extra_rows=(cr - 1, cr))
    assert "algo=tree" in d
    assert rel_err(got, ref) <= TOL


@pytest.mark.parametrize("n0,n1", [(64, 64), (64, 8), (16, 64), (64, 32)], ids=lambda v: str(v))
def test_tree_window64_complex(swd, orc, n0, n1):
    x = workloads.normal_complex((n0 + 150, n1 + 40), seed=900 + n0 + n1)
    got, ref, _ = run_sampled(swd, orc, x, n0, n1, "tree", seed=901)
    assert rel_err(got, ref) <= TOL


@pytest.mark.parametrize("wv", [1, 2])
def test_tree_64x32_waves_per_strip(swd, orc, monkeypatch, wv):
    """64 x 32 runs its split streams on one wave per strip by default and on
    two (four residues per stream) on request."""
    monkeypatch.setenv("SWDFT_TREE_WV", str(wv))
    x = workloads.normal_real((64 + 300, 32 + 20), seed=950)
    got, ref, d = run_sampled(swd, orc, x, 64, 32, "tree", seed=951)
    assert f"waves_per_strip={wv} " in d, d
    assert rel_err(got, ref) <= TOL


@pytest.mark.parametrize("n0,n1", [(64, 64), (64, 4), (8, 64)], ids=lambda v: str(v))
def test_swfft_window64(swd, orc, n0, n1):
    x = workloads.normal_real((n0 + 40, n1 + 70), seed=960 + n0 + n1)
    got, ref, d = run_sampled(swd, orc, x, n0, n1, "swfft", seed=961)
    assert "algo=swfft" in d
    assert rel_err(got, ref) <= TOL


def test_direct_f64_window64(swd, orc):
    """Full output (6 x 9 windows) of the FP64 direct kernel at 64 x 64."""
    x = workloads.normal_real((69, 72), seed=970).astype(np.float64)
    xt = torch.from_numpy(x).cuda()
    print("[case] direct_f64 64x64", flush=True)
    y = swd.swdft2d(xt, 64, 64, algo="direct_f64").cpu().numpy()
    assert rel_err(y, orc.swdft2d(x, 64, 64)) <= 1e-12


def test_fig4_image_all_algorithms_agree(swd):
    """The Fig. 4 setting: a 100 x 100 array with 64 x 64 windows through the
    tree, the per-window FFT and the FP64 direct kernel (on the same values
    widened exactly): FP32 paths within 1e-5 of the FP64 one."""
    x = workloads.normal_real((100, 100), seed=980)
    xt = torch.from_numpy(x).cuda()
    print("[case] fig4 100x100 64x64", flush=True)
    d = swd.swdft2d(xt.double(), 64, 64, algo="direct_f64").cpu().numpy()
    for algo in ("tree", "swfft"):
        y = swd.swdft2d(xt, 64, 64, algo=algo).cpu().numpy()
        assert rel_err(y, d) <= TOL, algo
