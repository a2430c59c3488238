"""Forward parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerance: normwise relative max error max|y_gpu - y_ref| / max|y_ref| <= 1e-5
for the FP32 tree (the target the workload states; the measured error is
~2e-7), <= 1e-12 for the FP64 direct kernel. Integer inputs with n_i <= 4 are
bit exact (every twiddle is a power of -i).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5
TOL_F64 = 1e-12


@pytest.fixture(scope="module")
def swd():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1707_08213_amd as swd
    return swd


def rel_err(got, ref):
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def gpu_full(swd, x_np, n0, n1, norm="none", algo="auto"):
    x = torch.from_numpy(np.ascontiguousarray(x_np)).cuda()
    print(f"[case] N={x_np.shape} n={n0}x{n1} dtype={x_np.dtype} norm={norm} algo={algo}",
          flush=True)
    y = swd.swdft2d(x, n0, n1, norm=norm, algo=algo)
    torch.cuda.synchronize()
    return y.cpu().numpy()


SHAPES = [(n0, n1) for n0 in (1, 2, 4, 8, 16, 32) for n1 in (1, 2, 4, 8, 16, 32)]


@pytest.mark.parametrize("n0,n1", SHAPES, ids=lambda v: str(v))
def test_tree_every_window_shape_real(swd, orc, n0, n1):
    # several strips and slabs plus ragged right and bottom tails
    N0 = 3 * n0 + 37
    N1 = 2 * (64 // n1) + n1 + 5
    x = workloads.normal_real((N0, N1), seed=100 + n0 * 64 + n1)
    y = gpu_full(swd, x, n0, n1)
    ref = orc.swdft2d(x.astype(np.float64), n0, n1)
    assert y.shape == ref.shape
    assert rel_err(y, ref) <= TOL_F32


@pytest.mark.parametrize("n0,n1", [(32, 8), (16, 16), (8, 32), (4, 2), (1, 16), (32, 1)],
                         ids=lambda v: str(v))
def test_tree_complex_input(swd, orc, n0, n1):
    x = workloads.normal_complex((2 * n0 + 29, 3 * (64 // n1) + n1 + 3), seed=7 + n0 + n1)
    y = gpu_full(swd, x, n0, n1)
    ref = orc.swdft2d(x.astype(np.complex128), n0, n1)
    assert rel_err(y, ref) <= TOL_F32


def test_tree_ortho_scale(swd, orc):
    x = workloads.normal_real((70, 90), seed=3)
    y = gpu_full(swd, x, 16, 8, norm="ortho")
    ref = orc.swdft2d(x.astype(np.float64), 16, 8, norm="ortho")
    assert rel_err(y, ref) <= TOL_F32
    y1 = gpu_full(swd, x, 16, 8)
    # n0 n1 = 128: the ortho scale is 2^-3.5, applied once to the row DFTs
    assert rel_err(y1 / np.sqrt(128.0), y) <= 1e-6


def test_tree_batched(swd, orc):
    x = workloads.normal_real((3, 41, 77), seed=9)
    xt = torch.from_numpy(x).cuda()
    y = swd.swdft2d(xt, 8, 16).cpu().numpy()
    for b in range(3):
        ref = orc.swdft2d(x[b].astype(np.float64), 8, 16)
        assert rel_err(y[b], ref) <= TOL_F32


def test_tree_exact_on_integer_fig3_shape(swd):
    """Fig. 3 shape (2 x 5 array, 2 x 4 windows) and a larger n <= 4 case with
    small integers: every twiddle is a power of -i, every partial sum is an
    exactly representable integer, so the FP32 tree must be bit exact."""
    rng = np.random.default_rng(5)
    for (N0, N1, n0, n1) in [(2, 5, 2, 4), (37, 53, 4, 4), (9, 70, 2, 2)]:
        x = rng.integers(-8, 9, size=(N0, N1)).astype(np.float32)
        y = gpu_full(swd, x, n0, n1)
        ref = oracle.swdft2d(x.astype(np.float64), n0, n1)
        assert np.array_equal(y.astype(np.complex128), ref)


def test_tree_whole_array_window(swd, orc):
    """N = n: one window, the plain 2D DFT of the array."""
    x = workloads.normal_real((32, 16), seed=4)
    y = gpu_full(swd, x, 32, 16)
    assert y.shape == (1, 1, 32, 16)
    assert rel_err(y[0, 0], np.fft.fft2(x.astype(np.float64))) <= TOL_F32


def test_tree_closed_forms(swd):
    """Impulse and constant inputs give their closed forms on the GPU too."""
    N0, N1, n0, n1 = 40, 50, 8, 16
    x = np.zeros((N0, N1), np.float32)
    r, c = 17, 23
    x[r, c] = 1.0
    y = gpu_full(swd, x, n0, n1)
    k0 = np.arange(n0)[:, None]
    k1 = np.arange(n1)[None, :]
    for q0 in range(N0 - n0 + 1):
        for q1 in range(N1 - n1 + 1):
            if q0 <= r < q0 + n0 and q1 <= c < q1 + n1:
                ref = np.exp(-2j * np.pi * ((r - q0) * k0 / n0 + (c - q1) * k1 / n1))
                assert np.max(np.abs(y[q0, q1] - ref)) < 1e-6
            else:
                assert np.all(y[q0, q1] == 0)
    y = gpu_full(swd, np.full((N0, N1), 2.0, np.float32), n0, n1)
    expect = np.zeros((n0, n1), complex)
    expect[0, 0] = 2.0 * n0 * n1
    assert np.max(np.abs(y - expect)) < 1e-5 * 2.0 * n0 * n1


def test_tree_deterministic(swd):
    x = torch.from_numpy(workloads.normal_real((300, 300), seed=8)).cuda()
    a = swd.swdft2d(x, 16, 16)
    b = swd.swdft2d(x, 16, 16)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(a), torch.view_as_real(b))


def test_direct_f64_small64(swd, orc):
    """64 x 64 real FP64, 4 x 4 windows: FP64 direct kernel against the oracle
    (<= 1e-12) and the FP32 tree on the FP32-rounded copy (<= 1e-5)."""
    w = workloads.small64()
    ref = orc.swdft2d(w["x"], 4, 4)
    y64 = gpu_full(swd, w["x"], 4, 4)
    assert y64.dtype == np.complex128
    assert rel_err(y64, ref) <= TOL_F64
    x32 = w["x"].astype(np.float32)
    y32 = gpu_full(swd, x32, 4, 4)
    assert rel_err(y32, orc.swdft2d(x32.astype(np.float64), 4, 4)) <= TOL_F32


@pytest.mark.parametrize("n0,n1,cplx", [(16, 16, False), (32, 8, True), (1, 32, False),
                                        (8, 1, True), (32, 32, False)])
def test_direct_f64_shapes(swd, orc, n0, n1, cplx):
    shape = (n0 + 19, n1 + 23)
    x = workloads.normal_complex(shape, 31, np.complex128) if cplx else \
        workloads.normal_real(shape, 31, np.float64)
    y = gpu_full(swd, x, n0, n1)
    assert rel_err(y, orc.swdft2d(x, n0, n1)) <= TOL_F64


def sampled_check(swd, orc, x_np, n0, n1, count, seed):
    x = torch.from_numpy(x_np).cuda()
    print(f"[case] full-size N={x_np.shape} n={n0}x{n1}", flush=True)
    y = swd.swdft2d(x, n0, n1)
    P0, P1 = x_np.shape[0] - n0 + 1, x_np.shape[1] - n1 + 1
    q0, q1 = workloads.window_sample(P0, P1, count, seed)
    got = y[torch.from_numpy(q0).cuda(), torch.from_numpy(q1).cuda()].cpu().numpy()
    xr = x_np.astype(np.complex128 if np.iscomplexobj(x_np) else np.float64)
    ref = orc.swdft2d(xr, n0, n1, windows=(q0, q1))
    del y
    torch.cuda.empty_cache()
    return got, ref


def test_sin1024_sampled(swd, orc):
    """1024 x 1024 real FP32 + 3 planted on-bin cosines, 16 x 16 windows:
    4096 sampled windows (corners and edges included) against the oracle, and
    the planted bins carry their amplitude."""
    w = workloads.sin1024()
    got, ref = sampled_check(swd, orc, w["x"], 16, 16, 4096, 1002)
    assert rel_err(got, ref) <= TOL_F32
    for (k0, k1, _ph) in w["planted"]:
        # each planted cosine puts 5*256/2 = 640 into bin (k0,k1); noise adds O(16)
        assert np.median(np.abs(got[:, k0, k1])) > 500


def test_cplx2048_sampled(swd, orc):
    """2048 x 512 complex64, 32 x 8 windows, 4096 sampled windows."""
    w = workloads.cplx2048()
    got, ref = sampled_check(swd, orc, w["x"], 32, 8, 4096, 1003)
    assert rel_err(got, ref) <= TOL_F32


def test_binding_rejects_bad_tensors(swd):
    p = swd.Plan(64, 64, 8, 8)
    with pytest.raises(ValueError):
        p.forward(torch.zeros(1, 64, 65, device="cuda"))
    with pytest.raises(ValueError):
        p.forward(torch.zeros(1, 64, 64, device="cuda", dtype=torch.float64))
    base = torch.zeros(1 + 64 * 64, device="cuda")
    with pytest.raises(swd.SwdftError) as e:
        p.exec_ptr(base.data_ptr() + 2, torch.empty(p.out_shape, dtype=torch.complex64,
                                                    device="cuda").data_ptr())
    assert e.value.name == "SWDFT_E_ALIGN"


@pytest.mark.parametrize("n0,n1,kg", [(8, 1, 2), (8, 8, 2), (8, 8, 1), (16, 16, 2), (16, 4, 2),
                                      (16, 8, 1), (32, 8, 1), (32, 32, 1), (32, 2, 2), (16, 32, 2),
                                      (8, 32, 1)],
                         ids=lambda v: str(v))
def test_tree_split_streams(swd, orc, n0, n1, kg):
    """Column streams split over kg lanes by k0 residue (per-lane twiddle
    rotation) must give the same transform as unsplit streams."""
    import os
    N0, N1 = 2 * n0 + 45, 3 * (64 // n1) + n1 + 1
    x = workloads.normal_complex((N0, N1), seed=n0 * 7 + n1 + kg)
    os.environ["SWDFT_TREE_KG"] = str(kg)
    try:
        y = gpu_full(swd, x, n0, n1)
    finally:
        del os.environ["SWDFT_TREE_KG"]
    assert rel_err(y, orc.swdft2d(x.astype(np.complex128), n0, n1)) <= TOL_F32


def _with_env(env, fn):
    import os
    saved = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return fn()
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("N0,N1,n0,n1,cplx,batch,env", [
    (70, 300, 16, 16, True, 3, {"SWDFT_TREE_WPC": 2}),
    (50, 200, 8, 8, False, 1, {"SWDFT_TREE_WPC": 1, "SWDFT_TREE_KG": 1}),
    (61, 150, 32, 8, False, 2, {"SWDFT_TREE_WPC": 1}),
    (90, 260, 16, 16, False, 1, {"SWDFT_TREE_WPC": 0, "SWDFT_TREE_SLAB": 16}),
    (70, 300, 32, 8, True, 2, {"SWDFT_TREE_WPC": 1, "SWDFT_TREE_WV": 2}),
    (45, 130, 16, 32, False, 1, {"SWDFT_TREE_WPC": 0, "SWDFT_TREE_WV": 2}),
    (80, 90, 32, 32, False, 1, {"SWDFT_TREE_WPC": 2, "SWDFT_TREE_WV": 2, "SWDFT_TREE_KG": 1}),
    (100, 140, 16, 8, True, 1, {"SWDFT_TREE_WPC": 1, "SWDFT_TREE_WV": 2, "SWDFT_TREE_KG": 2}),
], ids=["c16x16-b3-cap2", "r8x8-cap1-kg1", "r32x8-b2-cap1", "r16x16-nocap-slab16",
        "c32x8-b2-cap1-wv2", "r16x32-nocap-wv2", "r32x32-kg1-cap2-wv2", "c16x8-kg2-cap1-wv2"])
def test_tree_resident_cap(swd, orc, N0, N1, n0, n1, cplx, batch, env):
    """Launches capped at one or two resident workgroups per CU (padding
    LDS), uncapped ones, and strips shared by two waves compute the same
    transform."""
    gen = workloads.normal_complex if cplx else workloads.normal_real
    xs = np.stack([gen((N0, N1), seed=N0 + N1 + b) for b in range(batch)])
    dt = torch.complex64 if cplx else torch.float32

    def run():
        p = swd.Plan(N0, N1, n0, n1, dtype=dt, batch=batch)
        print(f"[case] {p.describe()}", flush=True)
        y = p.forward(torch.from_numpy(xs).cuda())
        torch.cuda.synchronize()
        return p.describe(), y.cpu().numpy()

    desc, y = _with_env(env, run)
    assert f"groups_per_cu={env['SWDFT_TREE_WPC']}" in desc
    if "SWDFT_TREE_WV" in env:
        assert f"waves_per_strip={env['SWDFT_TREE_WV']}" in desc
    for b in range(batch):
        ref = orc.swdft2d(xs[b].astype(np.complex128 if cplx else np.float64), n0, n1)
        assert rel_err(y[b], ref) <= TOL_F32, b


def test_tree_capped_dispatch_order_sampled(swd, orc):
    """One resident wave per CU with more tiles than one round of waves: the
    tiles run in dispatch order (rounds of contiguous strips)."""
    N0, N1 = 120, 1100
    x_np = workloads.normal_real((N0, N1), seed=77)

    def run():
        p = swd.Plan(N0, N1, 16, 16)
        return p.describe(), sampled_check(swd, orc, x_np, 16, 16, 2048, 1004)

    desc, (got, ref) = _with_env({"SWDFT_TREE_WPC": 1, "SWDFT_TREE_SLAB": 16}, run)
    assert "groups_per_cu=1" in desc and "order=dispatch" in desc, desc
    assert rel_err(got, ref) <= TOL_F32


@pytest.mark.parametrize("offset,count", [(0, 1 << 20), (1, (1 << 20) + 1), (1, 7), (0, 1)],
                         ids=["aligned", "head+tail", "short", "one"])
def test_write_probe_fills_exactly(swd, offset, count):
    """The write probe stores its constant into exactly the requested bytes,
    including an unaligned head and an odd tail."""
    buf = torch.zeros(count + 4, dtype=torch.complex64, device="cuda")
    start = buf.data_ptr() + 8 * offset
    from paper_1707_08213_amd import _lib
    _lib.check(_lib.lib.swdft2d_write_probe(start, 8 * count, None), "swdft2d_write_probe")
    torch.cuda.synchronize()
    v = torch.view_as_real(buf).cpu().numpy()
    inside = v[offset:offset + count]
    assert np.all(inside[:, 0] == 1.0) and np.all(inside[:, 1] == -1.0)
    assert np.all(v[:offset] == 0) and np.all(v[offset + count:] == 0)


@pytest.mark.parametrize("n0,n1", [(8, 8), (8, 16), (32, 16), (32, 32), (4, 16), (16, 4), (64, 8),
                                   (8, 64), (16, 8), (4, 4), (8, 32), (4, 8), (4, 32)],
                         ids=lambda v: str(v))
def test_default_launch_1024_sampled(swd, orc, n0, n1):
    """The default launch at 1024 x 1024 (caps of one or two workgroups per CU,
    whole streams or split, one or two waves per strip, as the plan picks):
    256 sampled windows, corners and edges included, against the oracle."""
    x = workloads.normal_real((1024, 1024), seed=1600 + n0 + n1)
    xt = torch.from_numpy(x).cuda()
    p = swd.Plan(1024, 1024, n0, n1)
    print(f"[case] {p.describe()}", flush=True)
    y = p.forward(xt.unsqueeze(0))[0]
    P0, P1 = 1024 - n0 + 1, 1024 - n1 + 1
    q0, q1 = workloads.window_sample(P0, P1, 256, 1601)
    got = y[torch.from_numpy(q0).cuda(), torch.from_numpy(q1).cuda()].cpu().numpy()
    del y
    torch.cuda.empty_cache()
    ref = orc.swdft2d(x.astype(np.float64), n0, n1, windows=(q0, q1))
    assert rel_err(got, ref) <= TOL_F32


@pytest.mark.parametrize("n0,n1,kg,wv,cplx", [
    (8, 1, 2, 2, False), (16, 1, 1, 2, False), (16, 1, 2, 2, True), (16, 2, 1, 2, False),
    (32, 1, 2, 2, False), (32, 1, 2, 2, True), (32, 2, 1, 2, True), (32, 2, 2, 2, False)],
    ids=lambda v: str(v))
def test_two_wave_first_chunk_repeatable(swd, orc, monkeypatch, n0, n1, kg, wv, cplx):
    """Two waves per strip share a chunk's row levels in LDS; with slabs of
    one or two rows every tile is mostly its first chunk, whose priming steps
    keep row values for the next chunk. Six launches must agree bitwise, and
    with the oracle (a read of a row after the other wave rewrote it would
    make them differ from run to run)."""
    monkeypatch.setenv("SWDFT_TREE_KG", str(kg))
    monkeypatch.setenv("SWDFT_TREE_WV", str(wv))
    N0, N1 = 3 * n0 + 37, 2 * (64 // n1) + n1 + 5
    x = (workloads.normal_complex((N0, N1), seed=1800 + n0 + n1) if cplx
         else workloads.normal_real((N0, N1), seed=1800 + n0 + n1))
    xt = torch.from_numpy(x).cuda()
    p = swd.Plan(N0, N1, n0, n1, dtype=xt.dtype)
    d = p.describe()
    print(f"[case] {d}", flush=True)
    assert f" kg={kg} " in d and f" waves_per_strip={wv} " in d, d
    y = torch.empty(p.out_shape, dtype=torch.complex64, device="cuda")
    runs = []
    for _ in range(6):
        y.fill_(float("nan"))
        p.forward(xt.unsqueeze(0), out=y)
        runs.append(y[0].cpu().numpy().copy())
    for r in runs[1:]:
        assert np.array_equal(r, runs[0])
    ref = orc.swdft2d(x.astype(np.complex128 if cplx else np.float64), n0, n1)
    assert rel_err(runs[0], ref) <= TOL_F32


@pytest.mark.parametrize("n0,n1,cplx", [(8, 16, True), (4, 8, False), (8, 32, False),
                                        (8, 8, True), (4, 16, False)], ids=lambda v: str(v))
def test_short_window_slabs_full(swd, orc, n0, n1, cplx):
    """Short windows in slabs of at most about 64 rows (ceil(P0 / 64) of
    them, two workgroups per CU) over a 200 x 400 image: every output against
    the oracle, the last slab ragged (193 or 197 window rows in 4 slabs)."""
    N0, N1 = 200, 400
    x = (workloads.normal_complex((N0, N1), seed=1700 + n0 + n1) if cplx
         else workloads.normal_real((N0, N1), seed=1700 + n0 + n1))
    xt = torch.from_numpy(x).cuda()
    p = swd.Plan(N0, N1, n0, n1, dtype=xt.dtype)
    d = p.describe()
    print(f"[case] {d}", flush=True)
    assert " slabs=4 " in d, d
    y = p.forward(xt.unsqueeze(0))[0].cpu().numpy()
    ref = orc.swdft2d(x.astype(np.complex128 if cplx else np.float64), n0, n1)
    assert y.shape == ref.shape
    assert rel_err(y, ref) <= TOL_F32


@pytest.mark.parametrize("n", [4, 8, 16, 32, 64])
def test_tree_fig4_size_short_slabs(swd, orc, n):
    """The Fig. 4 array size (100 x 100, square windows): small images take
    short slabs that are not whole chunks (the steps past a slab's last row
    are skipped) and split streams; real and complex input, a batch of two,
    against the oracle on every window."""
    x = workloads.normal_real((2, 100, 100), seed=900 + n)
    xc = workloads.normal_complex((100, 100), seed=950 + n)
    plan = swd.Plan(100, 100, n, n, torch.float32, batch=2)
    print(f"[case] fig4 size n={n} {plan.describe()}", flush=True)
    y = plan.forward(torch.from_numpy(x).cuda()).cpu().numpy()
    for b in range(2):
        assert rel_err(y[b], orc.swdft2d(x[b].astype(np.float64), n, n)) <= TOL_F32
    yc = gpu_full(swd, xc, n, n)
    assert rel_err(yc, orc.swdft2d(xc.astype(np.complex128), n, n)) <= TOL_F32


@pytest.mark.parametrize("count", [1 << 20, (1 << 20) + 1, 3, 1], ids=["large", "tail", "short", "one"])
def test_read_probe_reads_only(swd, count):
    """The read probe leaves its buffer and, for ordinary data, its sink
    untouched (an 8-byte tail included)."""
    buf = torch.randn(count, dtype=torch.complex64, device="cuda")
    before = buf.clone()
    sink = torch.full((1,), 42.0, dtype=torch.float32, device="cuda")
    from paper_1707_08213_amd import _lib
    _lib.check(_lib.lib.swdft2d_read_probe(buf.data_ptr(), 8 * count, sink.data_ptr(), None),
               "swdft2d_read_probe")
    torch.cuda.synchronize()
    assert torch.equal(buf, before)
    assert float(sink[0]) == 42.0
