"""Host-side checks of libswdft2d.so that need no GPU: the library loads, it
exports every entry point include/swdft2d.h declares, and plan validation /
argument checks return the documented status codes before anything is
enqueued (no call here reaches a kernel)."""
import ctypes
import json
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_lib = pytest.importorskip("paper_1707_08213_amd._lib",
                           reason="libswdft2d.so not built (python paper_1707_08213_amd/build.py)")
lib = _lib.lib
S = _lib.STATUS_CODE


def header_functions():
    text = open(os.path.join(ROOT, "include", "swdft2d.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(swdft[23]d_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = header_functions()
    assert "swdft2d_plan" in names and "swdft2d_exec" in names and "swdft2d_backward" in names
    assert "swdft3d_plan" in names and "swdft3d_exec" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in include/swdft2d.h but not exported"
        assert name in _lib.SIGNATURES, f"{name} has no ctypes signature in the binding"


def make_plan(N0, N1, n0, n1, dtype=_lib.SWDFT_R32, batch=1):
    h = ctypes.c_void_p()
    st = lib.swdft2d_plan(ctypes.byref(h), N0, N1, n0, n1, dtype, batch)
    return st, h


@pytest.mark.parametrize("args,status", [
    ((64, 64, 16, 16, 0, 1), "SWDFT_OK"),
    ((5, 2, 4, 2, 1, 3), "SWDFT_OK"),
    ((64, 64, 1, 1, 2, 1), "SWDFT_OK"),
    ((0, 64, 4, 4, 0, 1), "SWDFT_E_ARG"),
    ((64, 64, 4, 4, 0, 0), "SWDFT_E_ARG"),
    ((64, 64, 0, 4, 0, 1), "SWDFT_E_ARG"),
    ((64, 64, 4, 4, 7, 1), "SWDFT_E_ARG"),
    ((64, 64, 10, 4, 0, 1), "SWDFT_E_NOT_POW2"),
    ((64, 64, 4, 5, 0, 1), "SWDFT_E_NOT_POW2"),
    ((8, 64, 16, 4, 0, 1), "SWDFT_E_WINDOW"),
    ((128, 128, 64, 4, 0, 1), "SWDFT_OK"),
    ((100, 100, 64, 64, 0, 1), "SWDFT_OK"),
    ((256, 256, 128, 4, 0, 1), "SWDFT_E_WINDOW"),
    ((256, 256, 4, 128, 0, 1), "SWDFT_E_WINDOW"),
    ((1 << 40, 1 << 40, 32, 32, 0, 1), "SWDFT_E_OVERFLOW"),
    ((1 << 20, 1 << 20, 32, 32, 0, 1 << 20), "SWDFT_E_OVERFLOW"),
    ((64, 1 << 21, 16, 16, 1, 1), "SWDFT_OK"),            # longest row a plan accepts
    ((64, (1 << 21) + 1, 16, 16, 1, 1), "SWDFT_E_OVERFLOW"),
])
def test_plan_validation(args, status):
    st, h = make_plan(*args)
    assert _lib.STATUS[st] == status, lib.swdft2d_last_error()
    if st == 0:
        assert h.value is not None
        assert lib.swdft2d_destroy(h) == 0
    else:
        assert h.value is None
        assert lib.swdft2d_last_error()


def test_null_out_pointer():
    assert lib.swdft2d_plan(None, 8, 8, 2, 2, 0, 1) == S["SWDFT_E_ARG"]


def test_output_size_matches_paper_example():
    """Sec. 4.3: P0 = P1 = 400, n0 = n1 = 32 gives 163,840,000 complex numbers,
    2,621,440,000 bytes at 16 bytes each (complex128)."""
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))
    ex = g["output_size_example"]
    N0 = ex["P0"] + ex["n0"] - 1
    N1 = ex["P1"] + ex["n1"] - 1
    st, h = make_plan(N0, N1, ex["n0"], ex["n1"], _lib.SWDFT_R64)
    assert st == 0
    assert lib.swdft2d_output_elems(h) == ex["complex_numbers"]
    assert lib.swdft2d_output_bytes(h) == ex["bytes_complex128"]
    lib.swdft2d_destroy(h)
    st, h = make_plan(N0, N1, ex["n0"], ex["n1"], _lib.SWDFT_R32, 3)
    assert lib.swdft2d_output_elems(h) == 3 * ex["complex_numbers"]
    assert lib.swdft2d_output_bytes(h) == 3 * ex["complex_numbers"] * 8
    lib.swdft2d_destroy(h)


def test_fig3_shape_sizes():
    """Fig. 3: a 2 x 5 array with 2 x 4 windows has two window positions."""
    f = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))["fig3_shape"]
    st, h = make_plan(f["N0"], f["N1"], f["n0"], f["n1"])
    assert st == 0
    assert lib.swdft2d_output_elems(h) == f["windows"] * f["n0"] * f["n1"]
    lib.swdft2d_destroy(h)


def test_exec_argument_checks_do_not_launch():
    st, h = make_plan(64, 64, 16, 16)
    assert st == 0
    # null pointers
    assert lib.swdft2d_exec(h, None, 0x10000, None) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_exec(h, 0x10000, None, None) == S["SWDFT_E_ARG"]
    # misaligned input (float needs 4 bytes) and output (float2 needs 8 bytes)
    assert lib.swdft2d_exec(h, 0x10001, 0x90000000, None) == S["SWDFT_E_ALIGN"]
    assert lib.swdft2d_exec(h, 0x10000, 0x90000004, None) == S["SWDFT_E_ALIGN"]
    # overlapping input and output
    assert lib.swdft2d_exec(h, 0x10000, 0x10000 + 64, None) == S["SWDFT_E_ARG"]
    assert b"overlap" in lib.swdft2d_last_error()
    # backward: same checks with the roles swapped
    assert lib.swdft2d_backward(h, None, 0x10000, None) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_backward(h, 0x10004, 0x90000000, None) == S["SWDFT_E_ALIGN"]
    lib.swdft2d_destroy(h)


def test_destroyed_plan_is_rejected():
    st, h = make_plan(32, 32, 4, 4)
    assert lib.swdft2d_destroy(h) == 0
    assert lib.swdft2d_exec(h, 0x10000, 0x90000000, None) == S["SWDFT_E_PLAN"]
    assert lib.swdft2d_set_norm(h, 1) == S["SWDFT_E_PLAN"]
    assert lib.swdft2d_output_elems(h) == -1
    assert lib.swdft2d_destroy(h) == S["SWDFT_E_PLAN"]
    assert lib.swdft2d_destroy(None) == 0


def test_algo_dtype_rules():
    st, h = make_plan(32, 32, 4, 4, _lib.SWDFT_R32)
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_TREE) == 0
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_SWFFT) == 0
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_DIRECT_F64) == S["SWDFT_E_DTYPE"]
    assert lib.swdft2d_set_algo(h, 17) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_set_norm(h, 5) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_set_norm(h, 1) == 0
    lib.swdft2d_destroy(h)
    st, h = make_plan(32, 32, 4, 4, _lib.SWDFT_C64)
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_TREE) == S["SWDFT_E_DTYPE"]
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_SWFFT) == S["SWDFT_E_DTYPE"]
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_DIRECT_F64) == 0
    lib.swdft2d_destroy(h)


def test_describe_and_status_strings():
    st, h = make_plan(1024, 1024, 16, 16)
    buf = ctypes.create_string_buffer(256)
    assert lib.swdft2d_describe(h, buf, 256) == 0
    d = buf.value.decode()
    assert "algo=tree" in d and "n=16x16" in d
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_SWFFT) == 0
    assert lib.swdft2d_describe(h, buf, 256) == 0
    d = buf.value.decode()
    # 4 windows per 64-lane group, 253 groups per row: 33 slabs of 31 rows (>= 8192 groups)
    assert "algo=swfft" in d and "windows_per_group=4" in d, d
    rows = int(d.split("rows_per_group=")[1].split()[0])
    groups = int(d.split("groups=")[-1].split()[0])
    assert rows == 31 and groups == 253 * 33, d
    lib.swdft2d_destroy(h)
    for code, name in _lib.STATUS.items():
        assert lib.swdft2d_status_string(code).decode() == name
    assert lib.swdft2d_status_string(99) == b"SWDFT_E_UNKNOWN"


def test_read_probe_checks():
    assert lib.swdft2d_read_probe(None, 64, 0x20000, None) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_read_probe(0x10000, 64, None, None) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_read_probe(0x10000, 12, 0x20000, None) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_read_probe(0x10000, 0, 0x20000, None) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_read_probe(0x10008, 64, 0x20000, None) == S["SWDFT_E_ALIGN"]
    assert lib.swdft2d_read_probe(0x10000, 64, 0x20002, None) == S["SWDFT_E_ALIGN"]


def test_write_probe_checks():
    assert lib.swdft2d_write_probe(None, 64, None) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_write_probe(0x10000, 12, None) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_write_probe(0x10004, 16, None) == S["SWDFT_E_ALIGN"]


def make_batched(shapes, dtype=_lib.SWDFT_R32, offsets=None):
    descs = (_lib.Desc * len(shapes))()
    xo = yo = 0
    for i, (N0, N1, n0, n1) in enumerate(shapes):
        if offsets is not None:
            xo, yo = offsets[i]
        descs[i] = _lib.Desc(N0, N1, n0, n1, xo, yo)
        if offsets is None:
            xo += N0 * N1
            yo += (N0 - n0 + 1) * (N1 - n1 + 1) * n0 * n1
    h = ctypes.c_void_p()
    st = lib.swdft2d_plan_batched(ctypes.byref(h), ctypes.cast(descs, ctypes.c_void_p),
                                  len(shapes), dtype)
    return st, h


def test_batched_plan_validation():
    good = [(128, 256, 8, 8), (512, 128, 16, 16), (256, 256, 32, 32), (128, 512, 8, 32)]
    st, h = make_batched(good)
    assert st == 0, lib.swdft2d_last_error()
    expect = sum((a - c + 1) * (b - d + 1) * c * d for a, b, c, d in good)
    assert lib.swdft2d_output_elems(h) == expect
    buf = ctypes.create_string_buffer(1024)
    assert lib.swdft2d_describe(h, buf, 1024) == 0
    assert b"kind=batched" in buf.value and b"32x32" in buf.value
    # no adjoint for batched plans, and no FP64 algorithm
    assert lib.swdft2d_backward(h, 0x10000, 0x90000000, None) == S["SWDFT_E_PLAN"]
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_DIRECT_F64) == S["SWDFT_E_DTYPE"]
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_DENSE_BF16X2) == 0
    assert lib.swdft2d_tune(h, None, 0x10000, None) == S["SWDFT_E_ARG"]
    # x and y overlapping
    assert lib.swdft2d_exec(h, 0x10000, 0x10000 + 4096, None) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_destroy(h) == 0
    assert lib.swdft2d_plan_batched(None, None, 1, 0) == S["SWDFT_E_ARG"]
    st, _ = make_batched([])
    assert _lib.STATUS[st] == "SWDFT_E_ARG"
    cases = [
        ([(64, 64, 4, 8)], _lib.SWDFT_R32, "SWDFT_E_WINDOW"),     # 4 not in {8,16,32}
        ([(64, 64, 12, 8)], _lib.SWDFT_R32, "SWDFT_E_NOT_POW2"),
        ([(16, 64, 32, 8)], _lib.SWDFT_R32, "SWDFT_E_WINDOW"),    # n0 > N0
        ([(64, 64, 8, 8)], _lib.SWDFT_R64, "SWDFT_E_DTYPE"),
        ([(64, 64, 8, 8)], 9, "SWDFT_E_ARG"),
        ([(0, 64, 8, 8)], _lib.SWDFT_R32, "SWDFT_E_ARG"),
        ([(64, (1 << 21) + 1, 8, 8)], _lib.SWDFT_R32, "SWDFT_E_OVERFLOW"),  # row too long
    ]
    for shapes, dt, name in cases:
        st, h = make_batched(shapes, dt)
        assert _lib.STATUS[st] == name, (shapes, lib.swdft2d_last_error())
        assert h.value is None
    # negative and overlapping offsets
    st, _ = make_batched([(64, 64, 8, 8)], offsets=[(-1, 0)])
    assert _lib.STATUS[st] == "SWDFT_E_ARG"
    st, _ = make_batched([(64, 64, 8, 8), (64, 64, 8, 8)], offsets=[(0, 0), (4096, 100)])
    assert _lib.STATUS[st] == "SWDFT_E_ARG" and b"overlap" in lib.swdft2d_last_error()
    st, h = make_batched([(64, 64, 8, 8), (64, 64, 8, 8)], offsets=[(0, 0), (0, 57 * 57 * 64)])
    assert st == 0  # shared input, disjoint outputs
    lib.swdft2d_destroy(h)


def make_plan3(N, n, dtype=_lib.SWDFT_R32, batch=1):
    h = ctypes.c_void_p()
    st = lib.swdft3d_plan(ctypes.byref(h), *N, *n, dtype, batch)
    return st, h


@pytest.mark.parametrize("N,n,dtype,batch,status", [
    ((16, 16, 16), (8, 8, 8), _lib.SWDFT_R32, 1, "SWDFT_OK"),
    ((20, 9, 30), (16, 2, 4), _lib.SWDFT_C32, 3, "SWDFT_OK"),
    ((16, 16, 16), (8, 8, 8), _lib.SWDFT_R64, 1, "SWDFT_E_DTYPE"),
    ((16, 16, 16), (8, 8, 8), 7, 1, "SWDFT_E_ARG"),
    ((16, 0, 16), (8, 8, 8), _lib.SWDFT_R32, 1, "SWDFT_E_ARG"),
    ((16, 16, 16), (8, 8, 8), _lib.SWDFT_R32, 0, "SWDFT_E_ARG"),
    ((16, 16, 16), (8, 6, 8), _lib.SWDFT_R32, 1, "SWDFT_E_NOT_POW2"),
    ((16, 4, 16), (8, 8, 8), _lib.SWDFT_R32, 1, "SWDFT_E_WINDOW"),       # n1 > N1
    ((16, 16, 16), (32, 2, 2), _lib.SWDFT_R32, 1, "SWDFT_E_WINDOW"),     # n0 > N0
    ((64, 64, 64), (32, 2, 2), _lib.SWDFT_R32, 1, "SWDFT_E_WINDOW"),     # n0 outside {2..16}
    ((64, 64, 64), (4, 16, 2), _lib.SWDFT_R32, 1, "SWDFT_E_WINDOW"),     # n1 outside {2,4,8}
    ((64, 64, 64), (4, 2, 1), _lib.SWDFT_R32, 1, "SWDFT_E_WINDOW"),      # n2 outside {2,4,8}
    ((1 << 30, 1 << 30, 1 << 30), (8, 8, 8), _lib.SWDFT_R32, 1, "SWDFT_E_OVERFLOW"),
    ((1 << 16, 1 << 16, 40), (2, 2, 2), _lib.SWDFT_R32, 1, "SWDFT_E_OVERFLOW"),  # > 2^31 tiles
])
def test_plan3d_validation(N, n, dtype, batch, status):
    st, h = make_plan3(N, n, dtype, batch)
    assert _lib.STATUS[st] == status, lib.swdft2d_last_error()
    if st == 0:
        P = [N[i] - n[i] + 1 for i in range(3)]
        assert lib.swdft3d_output_elems(h) == batch * P[0] * P[1] * P[2] * n[0] * n[1] * n[2]
        buf = ctypes.create_string_buffer(512)
        assert lib.swdft3d_describe(h, buf, 512) == 0 and b"algo=tree3d" in buf.value
        assert lib.swdft3d_set_norm(h, 1) == 0
        assert lib.swdft3d_set_norm(h, 5) == S["SWDFT_E_ARG"]
        # argument checks before any launch
        assert lib.swdft3d_exec(h, None, 0x10000, None) == S["SWDFT_E_ARG"]
        assert lib.swdft3d_exec(h, 0x10002, 0x90000000, None) == S["SWDFT_E_ALIGN"]
        assert lib.swdft3d_exec(h, 0x10000, 0x90000004, None) == S["SWDFT_E_ALIGN"]
        assert lib.swdft3d_exec(h, 0x10000, 0x10000 + 64, None) == S["SWDFT_E_ARG"]  # overlap
        assert lib.swdft3d_destroy(h) == 0
        assert lib.swdft3d_destroy(h) == S["SWDFT_E_PLAN"]
        assert lib.swdft3d_output_elems(h) == -1
    else:
        assert h.value is None
    assert lib.swdft3d_plan(None, 8, 8, 8, 2, 2, 2, 0, 1) == S["SWDFT_E_ARG"]


def test_stream_validation():
    h = ctypes.c_void_p()
    cases = [
        ((64, 8, 8, _lib.SWDFT_R32), "SWDFT_OK"),
        ((64, 16, 32, _lib.SWDFT_C32), "SWDFT_OK"),
        ((0, 8, 8, _lib.SWDFT_R32), "SWDFT_E_ARG"),
        ((64, 8, 8, 9), "SWDFT_E_ARG"),
        ((64, 8, 8, _lib.SWDFT_R64), "SWDFT_E_DTYPE"),
        ((64, 6, 8, _lib.SWDFT_R32), "SWDFT_E_NOT_POW2"),
        ((4, 8, 8, _lib.SWDFT_R32), "SWDFT_E_WINDOW"),      # n1 > N1
        ((128, 64, 8, _lib.SWDFT_R32), "SWDFT_E_WINDOW"),   # n0 above 32
        (((1 << 21) + 1, 8, 8, _lib.SWDFT_R32), "SWDFT_E_OVERFLOW"),
    ]
    for args, name in cases:
        st = lib.swdft2d_stream_create(ctypes.byref(h), *args)
        assert _lib.STATUS[st] == name, (args, lib.swdft2d_last_error())
        if st == 0:
            N1, n0 = args[0], args[1]
            assert lib.swdft2d_stream_rows(h) == 0
            for R in (0, 1, n0 - 1, n0, 3 * n0 + 5):
                assert lib.swdft2d_stream_completes(h, R) == max(0, R - n0 + 1)
            assert lib.swdft2d_stream_completes(h, -1) == -1
            # argument errors are reported before anything touches a device
            assert lib.swdft2d_stream_push(h, 0x10000, -1, 0x90000000, None) == S["SWDFT_E_ARG"]
            assert lib.swdft2d_stream_push(h, 0x10000, 0, None, None) == 0  # no-op
            assert lib.swdft2d_stream_push(h, None, 4 * n0, 0x90000000, None) == S["SWDFT_E_ARG"]
            assert lib.swdft2d_stream_push(h, 0x10000, 4 * n0, None, None) == S["SWDFT_E_ARG"]
            assert lib.swdft2d_stream_push(h, 0x10002, 4 * n0, 0x90000000, None) == S["SWDFT_E_ALIGN"]
            assert lib.swdft2d_stream_push(h, 0x10000, 4 * n0, 0x90000004, None) == S["SWDFT_E_ALIGN"]
            assert lib.swdft2d_stream_push(h, 0x10000, 4 * n0, 0x10008, None) == S["SWDFT_E_ARG"]
            assert lib.swdft2d_stream_set_norm(h, 3) == S["SWDFT_E_ARG"]
            assert lib.swdft2d_stream_destroy(h) == 0
            assert lib.swdft2d_stream_destroy(h) == S["SWDFT_E_PLAN"]
            assert lib.swdft2d_stream_rows(h) == -1
        else:
            assert h.value is None
    assert lib.swdft2d_stream_create(None, 64, 8, 8, 0) == S["SWDFT_E_ARG"]
    assert lib.swdft2d_stream_push(None, 0x10000, 4, 0x90000000, None) == S["SWDFT_E_PLAN"]


@pytest.mark.parametrize("n0,n1,kg,cols,wv", [
    (64, 64, 1, 1, 2), (64, 32, 2, 1, 1), (64, 16, 4, 1, 1), (64, 8, 8, 1, 2), (64, 4, 8, 2, 2),
    (64, 1, 8, 8, 2), (32, 64, 1, 1, 1), (4, 64, 1, 1, 1)])
def test_window64_tree_shapes(n0, n1, kg, cols, wv):
    """n0 = 64 splits each stream over KG = min(8, 64/n1) lanes; 64 x 64, whose
    stream stays whole, the capped n1 <= 8 shapes and 64 x 1 (a small image
    here: 38 strips) run two waves per strip."""
    st, h = make_plan(200, 300, n0, n1)
    assert st == 0
    buf = ctypes.create_string_buffer(512)
    assert lib.swdft2d_describe(h, buf, 512) == 0
    d = buf.value.decode()
    assert f"kg={kg} " in d and f"cols_per_wave={cols} " in d and f"waves_per_strip={wv} " in d, d
    lib.swdft2d_destroy(h)


def test_window64_limits_of_other_paths():
    """Backward and streams stop at SWDFT_MAX_WINDOW_ADJ = 32, the dense variant
    at 32; the FP64 direct kernel and the per-window FFT take 64."""
    st, h = make_plan(100, 100, 64, 8)
    assert st == 0
    assert lib.swdft2d_backward(h, None, None, None) == S["SWDFT_E_WINDOW"]
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_DENSE_BF16X2) == S["SWDFT_E_WINDOW"]
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_SWFFT) == 0
    lib.swdft2d_destroy(h)
    st, h = make_plan(100, 100, 64, 64, _lib.SWDFT_R64)
    assert st == 0 and lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_DIRECT_F64) == 0
    lib.swdft2d_destroy(h)
    s = ctypes.c_void_p()
    assert lib.swdft2d_stream_create(ctypes.byref(s), 100, 64, 8, _lib.SWDFT_R32) == S["SWDFT_E_WINDOW"]
    assert lib.swdft2d_stream_create(ctypes.byref(s), 100, 8, 64, _lib.SWDFT_R32) == S["SWDFT_E_WINDOW"]
    assert lib.swdft2d_stream_create(ctypes.byref(s), 100, 32, 32, _lib.SWDFT_R32) == 0
    assert lib.swdft2d_stream_destroy(s) == 0


@pytest.mark.parametrize("N,n,slab,slabs", [
    (100, 16, 1, 85),     # one-chunk slabs: 22 strips x 85 slabs of 1 row, 1870 waves
    (100, 8, 1, 93),      # 12 strips x 93 slabs of 1 row
    (100, 32, 23, 3),     # 69 two-lane strips x 3 slabs: 207 workgroups (not whole chunks)
    (100, 64, 7, 6),      # 37 strips x 6 slabs of 7 rows: 222 workgroups
    (1024, 16, 1024, 1),  # one workgroup per CU walking whole columns
])
def test_tree_slab_rule(N, n, slab, slabs):
    """Small images (fewer tiles than compute units with one-chunk slabs;
    256 assumed without a device): for n0 <= 16 one chunk of rows per wave
    while the waves fit eight to a CU; otherwise the shortest slabs that keep
    to one workgroup per CU. Larger images keep their whole-column or
    about-4096-tile rules."""
    st, h = make_plan(N, N, n, n)
    assert st == 0
    buf = ctypes.create_string_buffer(512)
    assert lib.swdft2d_describe(h, buf, 512) == 0
    d = buf.value.decode()
    assert f" slab={slab} " in d and f" slabs={slabs} " in d, d
    lib.swdft2d_destroy(h)


@pytest.mark.parametrize("n0,n1,slab,slabs", [
    (8, 8, 64, 16), (8, 16, 64, 16), (8, 32, 64, 16), (4, 8, 64, 16), (4, 16, 64, 16),
    (4, 32, 1024, 1),   # measured slower in 64-row slabs: keeps the fewest slabs
    (4, 4, 128, 8),     # n1 = 4: the fewest slabs that fill the rounds
])
def test_tree_short_window_slab_rule(n0, n1, slab, slabs):
    """1024 x 1024 short windows: 8 x 8..32, 4 x 8 and 4 x 16 take 64-row
    slabs (two workgroups per CU on a device); 4 x 32 and n1 = 4 do not."""
    st, h = make_plan(1024, 1024, n0, n1)
    assert st == 0
    buf = ctypes.create_string_buffer(512)
    assert lib.swdft2d_describe(h, buf, 512) == 0
    d = buf.value.decode()
    assert f" slab={slab} " in d and f" slabs={slabs} " in d, d
    lib.swdft2d_destroy(h)


@pytest.mark.parametrize("N0,N1,n0,n1,dtype,batch,slab,slabs", [
    (1024, 1024, 16, 16, _lib.SWDFT_R32, 1, 1024, 1),   # one round of whole columns
    (1024, 1024, 16, 16, _lib.SWDFT_R32, 2, 48, 22),    # more rounds: 48-row slabs
    (256, 256, 16, 16, _lib.SWDFT_R32, 16, 48, 6),
    (2048, 2048, 16, 8, _lib.SWDFT_R32, 1, 64, 32),     # two-wave n1 = 8: 64-row slabs
    (2048, 2048, 32, 8, _lib.SWDFT_C32, 1, 64, 32),
    (1024, 1024, 64, 8, _lib.SWDFT_R32, 1, 128, 8),     # 64 rows rounded to a whole chunk
    (2048, 512, 32, 8, _lib.SWDFT_C32, 1, 1024, 2),     # one round: whole columns
])
def test_tree_multi_round_slab_rules(N0, N1, n0, n1, dtype, batch, slab, slabs):
    """Launches whose whole columns need more than one round of resident
    waves take short slabs (about 48 rows for 16 x 16, 64 for the two-wave
    n1 = 8 shapes, rounded up to whole chunks); one round keeps whole
    columns (256 compute units assumed without a device)."""
    st, h = make_plan(N0, N1, n0, n1, dtype, batch)
    assert st == 0
    buf = ctypes.create_string_buffer(512)
    assert lib.swdft2d_describe(h, buf, 512) == 0
    d = buf.value.decode()
    assert f" slab={slab} " in d and f" slabs={slabs} " in d, d
    lib.swdft2d_destroy(h)


def test_tree3d_slab_rule():
    """128^3 / 8 x 8 x 8: 32-row slabs at the resident cap."""
    st, h = make_plan3((128, 128, 128), (8, 8, 8))
    assert st == 0
    buf = ctypes.create_string_buffer(512)
    assert lib.swdft3d_describe(h, buf, 512) == 0
    d = buf.value.decode()
    assert " slab=32 " in d and " slabs=4 " in d, d
    lib.swdft3d_destroy(h)


@pytest.mark.parametrize("n0,n1,status", [
    (12, 9, "SWDFT_OK"), (24, 24, "SWDFT_OK"), (3, 16, "SWDFT_OK"), (8, 6, "SWDFT_OK"),
    (5, 4, "SWDFT_E_NOT_POW2"), (18, 3, "SWDFT_E_NOT_POW2"), (27, 3, "SWDFT_E_NOT_POW2"),
    (3, 2, "SWDFT_E_NOT_POW2"), (32, 3, "SWDFT_E_NOT_POW2"), (12, 64, "SWDFT_E_NOT_POW2")])
def test_mixed_radix_windows(n0, n1, status):
    """Sides from {3, 6, 9, 12, 24} pair with each other and with {4, 8, 16}."""
    st, h = make_plan(100, 100, n0, n1)
    assert st == S[status], (n0, n1, st)
    if st == 0:
        lib.swdft2d_destroy(h)


def test_mixed_radix_plan_rules():
    st, h = make_plan(200, 100, 24, 24)
    assert st == 0
    buf = ctypes.create_string_buffer(512)
    assert lib.swdft2d_describe(h, buf, 512) == 0
    d = buf.value.decode()
    # two 24-wide windows per wave (48 lanes), 32 rows per pass, ring period 12
    assert "radix=2,3" in d and " kg=1 " in d and " cols_per_wave=2 " in d, d
    assert " rows_per_chunk=96 " in d, d
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_SWFFT) == S["SWDFT_E_WINDOW"]
    assert lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_DENSE_BF16X2) == S["SWDFT_E_WINDOW"]
    assert lib.swdft2d_backward(h, None, None, None) == S["SWDFT_E_WINDOW"]
    lib.swdft2d_destroy(h)
    st, h = make_plan(100, 100, 12, 9, _lib.SWDFT_C64)
    assert st == 0 and lib.swdft2d_set_algo(h, _lib.SWDFT_ALGO_DIRECT_F64) == 0
    lib.swdft2d_destroy(h)
    s = ctypes.c_void_p()
    assert lib.swdft2d_stream_create(ctypes.byref(s), 100, 12, 8, _lib.SWDFT_R32) == \
        S["SWDFT_E_NOT_POW2"]


@pytest.mark.parametrize("N,n,kg,wv", [(100, 32, 2, 2), (100, 8, 1, 1), (100, 16, 1, 1),
                                       (100, 4, 1, 1), (100, 64, 1, 2),
                                       (1024, 32, 1, 2), (1024, 8, 2, 1)])
def test_tree_small_image_split(N, n, kg, wv):
    """Small images (fewer tiles than compute units) keep whole streams on one
    wave per strip for n0 <= 16 (one-chunk slabs), and split their streams
    over two lanes and two waves where those kernels exist for n0 = 32; large
    images keep the large-image defaults."""
    st, h = make_plan(N, N, n, n)
    assert st == 0
    buf = ctypes.create_string_buffer(512)
    assert lib.swdft2d_describe(h, buf, 512) == 0
    d = buf.value.decode()
    assert f" kg={kg} " in d and f" waves_per_strip={wv} " in d, d
    lib.swdft2d_destroy(h)


@pytest.mark.parametrize("n0,n1,slabs,waves", [
    (12, 16, 1, 253),    # strips fill one round of CUs: whole columns
    (24, 8, 2, 256),     # two slabs fill one round
    (12, 12, 5, 1015),   # capped at two per CU, slabs fill its rounds
    (9, 9, 7, 1022),     # uncapped, about 1024 tiles
])
def test_mixed_radix_launch_rules(n0, n1, slabs, waves):
    """Launch shapes of the mixed-radix tree at 1024 x 1024 (256 compute units
    assumed without a device; the resident cap itself needs a device)."""
    st, h = make_plan(1024, 1024, n0, n1)
    assert st == 0
    buf = ctypes.create_string_buffer(512)
    assert lib.swdft2d_describe(h, buf, 512) == 0
    d = buf.value.decode()
    assert f" slabs={slabs} " in d and f" waves={waves} " in d, d
    lib.swdft2d_destroy(h)


def _plan_twiddles(n0, n1):
    st, h = make_plan(max(n0, n1) + 8, max(n0, n1) + 8, n0, n1)
    assert st == S["SWDFT_OK"]
    try:
        out = []
        for axis, n in ((0, n0), (1, n1)):
            buf = (ctypes.c_float * (2 * n))()
            assert lib.swdft2d_twiddles(h, axis, buf, 2 * n) == S["SWDFT_OK"]
            out.append([(buf[2 * m], buf[2 * m + 1]) for m in range(n)])
        return out
    finally:
        lib.swdft2d_destroy(h)


def _rn_even_f32(exact):
    """Round an exact rational to the nearest float32, ties to even."""
    import numpy as np
    from fractions import Fraction
    f = np.float32(float(exact))
    best = None
    for c in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        d = abs(Fraction(float(c)) - exact)
        even = (int(np.array(c, dtype=np.float32).view(np.uint32)) & 1) == 0
        key = (d, not even)
        if best is None or key < best[0]:
            best = (key, c)
    return float(best[1])


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16, 32, 64, 3, 6, 9, 12, 24])
def test_fp32_twiddle_table(n):
    """Sec. 4.2's twiddle vectors as the kernels receive them: every entry is
    exp(-2 pi i m / n) rounded once to nearest-even FP32 (the exact value
    from 60-digit mpmath, rounded exactly here), 1 at m = 0 and -i at n/4
    exactly, and Omega[m + n/2] = -Omega[m] bit for bit for even n."""
    import struct
    from fractions import Fraction
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 60
    partner = 4 if n in (3, 6, 9, 12, 24) else n
    w0, w1 = _plan_twiddles(n, partner)
    w0b, w1b = _plan_twiddles(partner, n)
    assert w0 == w1b and w1 == w0b  # the same table on either axis
    table = w0

    def exact(v):  # 60 significant digits, far finer than any FP32 rounding boundary
        return Fraction(mpmath.nstr(v, 60, strip_zeros=False))

    for m in range(n):
        ang = -2 * mpmath.pi * m / n
        want = (_rn_even_f32(exact(mpmath.cos(ang))), _rn_even_f32(exact(mpmath.sin(ang))))
        assert table[m] == want, (n, m, table[m], want)
    assert table[0] == (1.0, 0.0)
    if n % 4 == 0:
        assert table[n // 4] == (0.0, -1.0)
        assert table[n // 2] == (-1.0, 0.0) and table[3 * n // 4] == (0.0, 1.0)
    if n % 2 == 0:
        bits = lambda v: struct.pack("<ff", *v)  # noqa: E731
        for m in range(n // 2):
            neg = (-table[m][0], -table[m][1])
            assert bits(table[m + n // 2]) == bits(neg), (n, m)


def test_twiddles_argument_checks():
    st, h = make_plan(40, 40, 8, 16)
    assert st == S["SWDFT_OK"]
    try:
        buf = (ctypes.c_float * 64)()
        assert lib.swdft2d_twiddles(h, 2, buf, 64) == S["SWDFT_E_ARG"]
        assert lib.swdft2d_twiddles(h, 1, buf, 31) == S["SWDFT_E_ARG"]
        assert lib.swdft2d_twiddles(h, 0, None, 64) == S["SWDFT_E_ARG"]
        assert lib.swdft2d_twiddles(h, 1, buf, 32) == S["SWDFT_OK"]
    finally:
        lib.swdft2d_destroy(h)
    assert lib.swdft2d_twiddles(None, 0, buf, 64) == S["SWDFT_E_PLAN"]


def test_every_environment_variable_is_documented():
    """Each environment variable the library reads appears in the header's
    list of environment variables."""
    import glob
    names = set()
    for path in glob.glob(os.path.join(ROOT, "paper_1707_08213_amd", "csrc", "*.hip")):
        text = open(path).read()
        names |= set(re.findall(r'(?:getenv|env_int)\(\s*"(SWDFT[A-Z0-9_]*)"', text))
    assert "SWDFT_TREE_KG" in names and "SWDFT_AUTOTUNE_CACHE" in names
    header = open(os.path.join(ROOT, "include", "swdft2d.h")).read()
    missing = sorted(n for n in names if not re.search(r"\*\s+" + n + r"\s", header))
    assert not missing, f"environment variables read but not documented: {missing}"
