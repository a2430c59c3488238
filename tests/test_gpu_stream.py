"""Streaming 2D SWDFT (the real-time order of Sec. 4.3): rows pushed in
chunks of any size give, concatenated, the transform of the whole image,
against the FP64 oracle (<= 1e-5) and against a single-plan launch with the
same split of each stream (<= 1e-6: the two kernels run the same node
operations, but the compiler may fuse multiply-adds differently in each)."""
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


def stream_all(swd, x_np, n0, n1, chunks, norm="none"):
    s = swd.Stream2D(x_np.shape[1], n0, n1, dtype=torch.from_numpy(x_np[:1]).dtype, norm=norm)
    x = torch.from_numpy(x_np).cuda()
    outs, r = [], 0
    for c in chunks:
        outs.append(s.push(x[r:r + c].contiguous()))
        r += c
    assert r == x_np.shape[0] and s.rows == r
    torch.cuda.synchronize()
    y = torch.cat(outs) if outs else None
    return s, y


def single_plan_kg1(swd, x_np, n0, n1, norm="none"):
    saved = {k: os.environ.get(k) for k in ("SWDFT_TREE_KG", "SWDFT_TREE_WV")}
    os.environ["SWDFT_TREE_KG"] = "1"
    os.environ["SWDFT_TREE_WV"] = "1"
    try:
        return swd.swdft2d(torch.from_numpy(x_np).cuda(), n0, n1, norm=norm)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def chunk_list(total, seed):
    rng = np.random.default_rng(seed)
    out, r = [], 0
    while r < total:
        c = int(rng.choice([1, 2, 3, 5, 7, 16, 29, 64]))
        c = min(c, total - r)
        out.append(c)
        r += c
    return out


SHAPES = [(1, 8), (2, 4), (4, 16), (8, 8), (8, 32), (16, 16), (16, 1), (32, 8), (32, 32), (4, 2)]


@pytest.mark.parametrize("n0,n1", SHAPES, ids=lambda v: str(v))
def test_stream_matches_oracle_and_single_plan(swd, orc, n0, n1):
    N0, N1 = 3 * n0 + 45, 2 * (64 // n1) + n1 + 3
    x = workloads.normal_real((N0, N1), seed=500 + n0 * 64 + n1)
    chunks = chunk_list(N0, n0 * 100 + n1)
    print(f"[case] stream n={n0}x{n1} N={N0}x{N1} chunks={chunks[:8]}...", flush=True)
    _, y = stream_all(swd, x, n0, n1, chunks)
    ref = orc.swdft2d(x.astype(np.float64), n0, n1)
    got = y.cpu().numpy()
    assert got.shape == ref.shape
    assert rel_err(got, ref) <= TOL
    single = single_plan_kg1(swd, x, n0, n1).cpu().numpy()
    assert rel_err(got, single) <= 1e-6


def test_stream_complex_ortho_and_reset(swd, orc):
    n0, n1 = 8, 16
    x = workloads.normal_complex((70, 90), seed=9)
    s, y = stream_all(swd, x, n0, n1, [3, 9, 1, 40, 17], norm="ortho")
    ref = orc.swdft2d(x.astype(np.complex128), n0, n1, norm="ortho")
    assert rel_err(y.cpu().numpy(), ref) <= TOL
    # after reset the same rows give the same output, pushed differently
    s.reset()
    assert s.rows == 0
    xt = torch.from_numpy(x).cuda()
    y2 = torch.cat([s.push(xt[:35].contiguous()), s.push(xt[35:].contiguous())])
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(y2), torch.view_as_real(y))


@pytest.mark.parametrize("n0,n1", [(4, 4), (4, 16), (2, 8), (16, 4)], ids=lambda v: str(v))
def test_stream_complex_split_streams(swd, orc, n0, n1):
    """Complex input through the split streams of small n0 (from n0 = 4 on a
    stream spans two lanes): random push sizes against the oracle."""
    x = workloads.normal_complex((2 * n0 + 41, 3 * (64 // n1) + n1 + 2), seed=610 + 8 * n0 + n1)
    chunks = chunk_list(x.shape[0], 7 * n0 + n1)
    print(f"[case] complex stream n={n0}x{n1} chunks={chunks[:8]}...", flush=True)
    _, y = stream_all(swd, x, n0, n1, chunks)
    ref = orc.swdft2d(x.astype(np.complex128), n0, n1)
    assert rel_err(y.cpu().numpy(), ref) <= TOL


def test_stream_short_pushes_emit_nothing_until_a_window_completes(swd):
    n0, n1 = 16, 8
    s = swd.Stream2D(40, n0, n1)
    x = torch.randn(n0 + 2, 40, device="cuda")
    counts = [s.push(x[i:i + 1].contiguous()).shape[0] for i in range(n0 + 2)]
    assert counts == [0] * (n0 - 1) + [1, 1, 1]


def test_sin1024_streamed_sampled(swd, orc):
    """sin1024 streamed in pushes of 37 rows: sampled windows against the oracle."""
    w = workloads.sin1024()
    x = w["x"]
    _, y = stream_all(swd, x, 16, 16, [37] * (1024 // 37) + [1024 % 37])
    P0, P1 = 1009, 1009
    q0, q1 = workloads.window_sample(P0, P1, 1024, 1005)
    got = y[torch.from_numpy(q0).cuda(), torch.from_numpy(q1).cuda()].cpu().numpy()
    del y
    torch.cuda.empty_cache()
    ref = orc.swdft2d(x.astype(np.float64), 16, 16, windows=(q0, q1))
    assert rel_err(got, ref) <= TOL
