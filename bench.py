"""Throughput of the 2D Tree SWDFT hot path on one MI355X.

Default workload (``--workload sin1024``): one 1024 x 1024 real FP32 image
(N(0,1) plus three planted on-bin 2D cosines of amplitude 5), 16 x 16
windows -> 1009 x 1009 x 256 complex64 coefficients (2.085 GB) per step. A
step is one forward transform through the C ABI with x and y resident in HBM.

Prints one JSON line: coefficients/s of the FP32 tree, the roofline of its
kernel (HBM-bound: algorithmic bytes = complex64 output + input per launch,
over the average launch duration from HIP events on the launch stream), the
FP64 direct form timed on the same GPU, a write-only probe at the same byte
count, the normwise relative error on sampled windows, and the FP64 oracle
timed on the host cores on a bounded sample of the same windows.

Other workloads (one JSON line each, same fields where they apply):
  cplx2048 - 2048 x 512 complex64, 32 x 8 windows (tree; dense MFMA variant;
             adjoint).
  grad256  - 16 x 256 x 256 real FP32, 16 x 16 windows, forward + adjoint of
             L = sum w |A|^2 (band mask w); the adjoint kernel is read-bound.
  The adjoint legs also time a read-only probe over dy (the read ceiling at
  the same byte count).
  uneven64 - 64 real FP32 images of uneven sizes and window shapes in one
             batched graph launch, after autotuning.
  mixed1024 - 1024 x 1024 real FP32, 12 x 12 windows through the mixed-radix
             (2 and 3) tree; 9 x 9, 24 x 24 and 12 x 16 as extra lines.

``--fig4`` runs the speed comparison of Fig. 4 instead (a markdown table, no
JSON line): square windows n = 4..64 over a 100 x 100 real array, and over a
1024 x 1024 one, through the FP64 direct form of Eq. (2), the per-window FFT
and the tree.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
import statistics

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SWDFT coeffs/s + % HBM roofline, FP32 tree vs plain FP64 direct @ rel err≤1e-5"
PEAK_HBM_GBS = 8000.0
# the kernel and the host code that picks its launch shape (tile, occupancy cap)
KERNEL_SOURCES = ["paper_1707_08213_amd/csrc/tree_fwd_kernel.h",
                  "paper_1707_08213_amd/csrc/tree_fwd_n16_r_16.hip",
                  "paper_1707_08213_amd/csrc/tree_fwd.hip",
                  "paper_1707_08213_amd/csrc/tree_config.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tree_fwd_sin1024_traffic.json")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def code_only(text: str) -> str:
    """C++ source without comments and with whitespace runs collapsed, so that
    editing a comment does not invalidate recorded counters."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_hash(read=None) -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        if read is None:
            with open(os.path.join(ROOT, p), encoding="utf-8") as f:
                text = f.read()
        else:
            text = read(p)
        h.update(code_only(text).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def pmc_summary(fetch_db: str, write_db: str, copy_bytes: int, out_json: str) -> str:
    """Turn two rocprofv3 --pmc databases (FETCH_SIZE, then WRITE_SIZE, KiB per
    dispatch) into per-kernel HBM bytes. Each counter is scaled by what it reads
    for the runtime's plain device copy of `copy_bytes` bytes (run by
    --copy-calibration). Writes the tree kernel's bytes per launch, tagged with
    the hash of its source, to `out_json`; returns a markdown table."""
    import collections
    import sqlite3
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for path, counter in ((fetch_db, "FETCH_SIZE"), (write_db, "WRITE_SIZE")):
        con = sqlite3.connect(path)
        for name, v in con.execute("select kernel_name, value from counters_collection "
                                   "where counter_name = ?", (counter,)):
            vals[name][counter].append(float(v))
        con.close()
    copy = [k for k in vals if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no device copy kernel in the counter databases")
    kib = copy_bytes / 1024.0

    def mean(xs):
        return sum(xs) / len(xs)

    f_scale = kib / mean(vals[copy[0]]["FETCH_SIZE"])
    w_scale = kib / mean(vals[copy[0]]["WRITE_SIZE"])
    lines = ["| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM read B | HBM write B |",
             "|---|---|---|---|---|---|"]
    tree_bytes = None
    for name, c in sorted(vals.items()):
        f, w = mean(c["FETCH_SIZE"]), mean(c["WRITE_SIZE"])
        rb, wb = f * f_scale * 1024, w * w_scale * 1024
        short = name.replace("(anonymous namespace)", "anon").split("(")[0][:60]
        lines.append(f"| {short} | {len(c['FETCH_SIZE'])} | {f:.1f} | {w:.1f} | {rb:.4g} | {wb:.4g} |")
        if "tree_fwd_kernel<16, 16, true" in name:
            tree_bytes = rb + wb
    lines.append("")
    lines.append(f"copy reference: {copy_bytes} B read and written; scale FETCH x{f_scale:.4f}, "
                 f"WRITE x{w_scale:.4f}")
    if tree_bytes is not None:
        with open(out_json, "w") as fh:
            json.dump({"kernel": "tree_fwd_kernel<16,16,real>", "workload": "sin1024",
                       "kernel_hash": kernel_hash(), "hbm_bytes_per_launch": tree_bytes,
                       "fetch_scale": f_scale, "write_scale": w_scale}, fh, indent=1)
            fh.write("\n")
    return "\n".join(lines)


def counter_summary(db: str) -> str:
    """Per-kernel means of every counter in a rocprofv3 --pmc database
    (markdown), and each SQ_INSTS_* / SQ_WAIT_* counter divided by SQ_WAVES
    when that counter was collected (per-wave figures)."""
    import collections
    import sqlite3
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    con = sqlite3.connect(db)
    for name, counter, v in con.execute(
            "select kernel_name, counter_name, value from counters_collection"):
        short = name.replace("(anonymous namespace)", "anon").split("(")[0].replace("void ", "")
        vals[short][counter].append(float(v))
    con.close()
    counters = sorted({c for d in vals.values() for c in d})
    lines = ["| kernel | dispatches | " + " | ".join(counters) + " |",
             "|---|---|" + "---|" * len(counters)]
    per_wave = []
    for name, d in sorted(vals.items()):
        n = max(len(v) for v in d.values())
        means = {c: sum(d[c]) / len(d[c]) for c in counters if d.get(c)}
        lines.append(f"| {name[:70]} | {n} | " +
                     " | ".join(f"{means[c]:.4g}" if c in means else "" for c in counters) + " |")
        if means.get("SQ_WAVES"):
            w = means["SQ_WAVES"]
            per_wave.append((name, w, {c: means[c] / w for c in means
                                       if c.startswith(("SQ_INSTS", "SQ_WAIT", "SQ_WAVE_CYCLES",
                                                        "SQ_BUSY"))}))
    if per_wave:
        cols = sorted({c for _, _, d in per_wave for c in d})
        lines += ["", "Per wave (counter / SQ_WAVES):", "",
                  "| kernel | waves | " + " | ".join(cols) + " |",
                  "|---|---|" + "---|" * len(cols)]
        for name, w, d in per_wave:
            lines.append(f"| {name[:70]} | {w:.0f} | " +
                         " | ".join(f"{d[c]:.4g}" if c in d else "" for c in cols) + " |")
    return "\n".join(lines)


def trace_summary(db: str) -> str:
    """Per-kernel duration table (markdown) from a rocprofv3 --kernel-trace
    database, one row per kernel and grid size."""
    import collections
    import sqlite3
    import statistics
    con = sqlite3.connect(db)
    durs = collections.defaultdict(list)
    meta = {}
    for name, dur, gx, wx, lds in con.execute(
            "select name, duration, grid_x, workgroup_x, lds_size from kernels"):
        short = name.replace("(anonymous namespace)", "anon").split("(")[0].replace("void ", "")
        key = (short, gx // max(wx, 1))
        durs[key].append(dur / 1000.0)
        meta[key] = (wx, lds)
    con.close()
    lines = ["| kernel | calls | avg us | min us | max us | workgroups x size | LDS B |",
             "|---|---|---|---|---|---|---|"]
    for key, v in sorted(durs.items(), key=lambda kv: -sum(kv[1])):
        wx, lds = meta[key]
        lines.append(f"| {key[0][:75]} | {len(v)} | {statistics.mean(v):.1f} | {min(v):.1f} | "
                     f"{max(v):.1f} | {key[1]} x {wx} | {lds} |")
    return "\n".join(lines)


def time_launches(fn, steps: int, stream):
    """Average per-launch duration (ms) from event pairs on `stream`, and the
    wall time of the whole loop (s), bracketed by device synchronisation."""
    import torch
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        fn()
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    durs = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return sum(durs) / len(durs), wall, durs


def time_batch(fn, steps: int, stream) -> float:
    """Average duration (ms) of `steps` back-to-back calls from one event
    pair on `stream`."""
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / steps


def roofline(alg_bytes: int, avg_ms: float, kernel: str, traffic=None, med_ms=None) -> dict:
    """`achieved` uses the mean launch duration; the median is reported beside
    it (and the fraction it gives)."""
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": achieved / PEAK_HBM_GBS, "traffic": traffic, "kernel": kernel,
           "algorithmic_bytes_per_launch": alg_bytes, "avg_launch_us": avg_ms * 1e3}
    if med_ms is not None:
        out["median_launch_us"] = med_ms * 1e3
        out["median_frac"] = alg_bytes / (med_ms * 1e-3) / 1e9 / PEAK_HBM_GBS
    return out


def oracle_rate(orc, x2d, n0, n1, P0, P1, seconds: float, seed: int):
    """Time the oracle on a seeded window sample sized to about `seconds`."""
    import workloads
    q0, q1 = workloads.window_sample(P0, P1, 256, seed)
    t0 = time.perf_counter()
    orc.swdft2d(x2d, n0, n1, windows=(q0, q1))
    per_win = (time.perf_counter() - t0) / q0.size
    nwin = int(min(P0 * P1, max(512, seconds / per_win)))
    s0, s1 = workloads.window_sample(P0, P1, nwin, seed + 1)
    t0 = time.perf_counter()
    orc.swdft2d(x2d, n0, n1, windows=(s0, s1))
    dt = time.perf_counter() - t0
    out = {"value": s0.size * n0 * n1 / dt, "unit": "coeffs/s", "cores": orc.num_threads(),
           "kind": "oracle",
           "sample": f"{s0.size} of the {P0}x{P1} windows (seeded, corners and edges "
                     f"included), {s0.size * n0 * n1} coefficients in {dt:.1f} s"}
    # the same code on one host core, on about a tenth of the time budget
    threads = orc.num_threads()
    orc.set_threads(1)
    try:
        n1c = int(min(s0.size, max(64, 0.1 * seconds / (per_win * threads))))
        c0, c1 = workloads.window_sample(P0, P1, n1c, seed + 2)
        t0 = time.perf_counter()
        orc.swdft2d(x2d, n0, n1, windows=(c0, c1))
        dt1 = time.perf_counter() - t0
    finally:
        orc.set_threads(threads)
    out["one_core"] = {"value": c0.size * n0 * n1 / dt1, "unit": "coeffs/s",
                       "sample": f"{c0.size} windows in {dt1:.1f} s"}
    return out


def base_record(args, value, ms_per_step, dtype, config) -> dict:
    return {"metric": METRIC, "value": value, "unit": "coeffs/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def forward_leg(plan, x, args, stream):
    """Warm up and time `plan.forward`; returns (y, avg_ms, wall_per_step_s,
    median_ms)."""
    import torch
    y = torch.empty(plan.out_shape, dtype=plan.out_dtype, device=x.device)
    for _ in range(args.warmup):
        plan.forward(x, out=y)
    torch.cuda.synchronize()
    avg_ms, wall, durs = time_launches(lambda: plan.forward(x, out=y), args.steps, stream)
    return y, avg_ms, wall / args.steps, statistics.median(durs)


def sampled(y_img, q0, q1):
    import torch
    dev = y_img.device
    return y_img[torch.from_numpy(q0).to(dev), torch.from_numpy(q1).to(dev)].cpu().numpy()


def rel(a, b):
    import numpy as np
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def run_sin1024(args, swd, dev) -> dict:
    import numpy as np
    import torch

    import workloads
    wl = workloads.sin1024()
    x_np = wl["x"]
    N0, N1 = x_np.shape
    n0, n1 = wl["n0"], wl["n1"]
    P0, P1 = N0 - n0 + 1, N1 - n1 + 1
    x = torch.from_numpy(x_np).to(dev).unsqueeze(0)
    plan = swd.Plan(N0, N1, n0, n1, torch.float32, batch=1)
    coeffs = plan.output_elems()
    alg_bytes = plan.output_bytes() + x.numel() * 4
    stream = torch.cuda.current_stream(dev)
    log(plan.describe())
    if args.copy_calibration:
        src = torch.ones(plan.output_bytes() // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: 3 copies of {src.numel() * 4} bytes")
        del src, dst
    y, avg_ms, step_s, med_ms = forward_leg(plan, x, args, stream)
    rf = roofline(alg_bytes, avg_ms, "tree_fwd_kernel<16,16,real>", measured_traffic(), med_ms)
    log(f"tree: {avg_ms * 1e3:.1f} us/launch, {rf['achieved']:.0f} GB/s")
    q0, q1 = workloads.window_sample(P0, P1, 4096, 2002)
    got = sampled(y[0], q0, q1)

    swd.write_probe(y)
    torch.cuda.synchronize()
    probe_ms, _, _ = time_launches(lambda: swd.write_probe(y), 10, stream)
    probe_gbs = plan.output_bytes() / (probe_ms * 1e-3) / 1e9
    del y

    comparator, got64 = None, None
    if not args.no_comparator:
        x64 = x.double()
        p64 = swd.Plan(N0, N1, n0, n1, torch.float64, batch=1, algo="direct_f64")
        y64 = torch.empty(p64.out_shape, dtype=torch.complex128, device=dev)
        p64.forward(x64, out=y64)
        torch.cuda.synchronize()
        d_ms, d_wall, _ = time_launches(lambda: p64.forward(x64, out=y64), 3, stream)
        got64 = sampled(y64[0], q0, q1)
        comparator = {"algo": "direct_f64", "value": coeffs / (d_wall / 3), "unit": "coeffs/s",
                      "ms_per_step": d_wall / 3 * 1e3, "avg_launch_ms": d_ms, "dtype": "f64",
                      "tree_speedup": (d_wall / 3) / step_s}
        del y64, x64
        torch.cuda.empty_cache()
        log(f"direct_f64: {d_ms:.2f} ms/launch")

    cpu, err = None, None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.get()
        xd = x_np.astype(np.float64)
        ref = orc.swdft2d(xd, n0, n1, windows=(q0, q1))
        err = rel(got, ref)
        if got64 is not None:
            comparator["rel_err"] = rel(got64, ref)
        cpu = oracle_rate(orc, xd, n0, n1, P0, P1, args.cpu_seconds, 3002)
        log(f"oracle: {cpu['value']:.3e} coeffs/s on {cpu['cores']} threads")

    out = base_record(args, coeffs / step_s, step_s * 1e3, "f32", {
        "workload": "sin1024: one 1024x1024 real FP32 image, N(0,1) + 3 planted on-bin "
                    "2D cosines (amplitude 5), 16x16 windows, stride 1 -> "
                    "1009x1009x256 complex64 coefficients",
        "N0": N0, "N1": N1, "n0": n0, "n1": n1, "batch": 1, "algo": "tree",
        "coeffs_per_step": coeffs})
    out.update({"roofline": rf, "rel_err": err,
                "write_probe": {"GB/s": probe_gbs, "frac": probe_gbs / PEAK_HBM_GBS,
                                "bytes": plan.output_bytes()},
                "comparator": comparator, "cpu_baseline": cpu})
    return out


def run_cplx2048(args, swd, dev) -> dict:
    import numpy as np
    import torch

    import workloads
    wl = workloads.cplx2048()
    x_np = wl["x"]
    N0, N1 = x_np.shape
    n0, n1 = wl["n0"], wl["n1"]
    P0, P1 = N0 - n0 + 1, N1 - n1 + 1
    x = torch.from_numpy(x_np).to(dev).unsqueeze(0)
    plan = swd.Plan(N0, N1, n0, n1, torch.complex64, batch=1)
    coeffs = plan.output_elems()
    alg_bytes = plan.output_bytes() + x.numel() * 8
    stream = torch.cuda.current_stream(dev)
    log(plan.describe())
    y, avg_ms, step_s, med_ms = forward_leg(plan, x, args, stream)
    rf = roofline(alg_bytes, avg_ms, "tree_fwd_kernel<32,8,complex>", med_ms=med_ms)
    log(f"tree: {avg_ms * 1e3:.1f} us/launch, {rf['achieved']:.0f} GB/s")
    q0, q1 = workloads.window_sample(P0, P1, 4096, 2003)
    got = sampled(y[0], q0, q1)
    # the dense matrix-core variant on the same input and output buffer
    pd = swd.Plan(N0, N1, n0, n1, torch.complex64, batch=1, algo="dense_bf16x2")
    log(pd.describe())
    for _ in range(args.warmup):
        pd.forward(x, out=y)
    torch.cuda.synchronize()
    d_ms, d_wall, _ = time_launches(lambda: pd.forward(x, out=y), args.steps, stream)
    got_d = sampled(y[0], q0, q1)
    # real flops of the three split products, times 3: per window position, the
    # row product of its one new input row (n1 x n1; the n0 windows that read
    # a row share it) and the n0 x n0 column product over n1 columns,
    # 8 n1 (n1 + n0^2) (priming rows of a slab not counted)
    d_flops = 3 * 8 * n1 * (n1 + n0 * n0) * P0 * P1
    dense = {"algo": "dense_bf16x2", "value": coeffs / (d_wall / args.steps), "unit": "coeffs/s",
             "avg_launch_us": d_ms * 1e3,
             "roofline": roofline(alg_bytes, d_ms, "dense_fwd_kernel<32,8,complex>"),
             "mfma_tflops": d_flops / (d_ms * 1e-3) / 1e12, "mfma_peak_tflops": 2500.0}
    log(f"dense: {d_ms * 1e3:.1f} us/launch")
    # the adjoint (transposed tree) of the same plan: reads dy (the layout of
    # y; here the dense output), writes dx
    dx = torch.empty_like(x)
    for _ in range(args.warmup):
        plan.backward(y, out=dx)
    torch.cuda.synchronize()
    a_ms, _, a_durs = time_launches(lambda: plan.backward(y, out=dx), args.steps, stream)
    adj = {"roofline": roofline(plan.output_bytes() + x.numel() * 8, a_ms,
                                "tree_adj_kernel<32,8,complex> + reduce",
                                med_ms=statistics.median(a_durs)),
           "avg_launch_us": a_ms * 1e3}
    adj["read_probe"] = read_probe_leg(swd, y, stream)
    log(f"adjoint: {a_ms * 1e3:.1f} us/launch ({adj['roofline']['achieved']:.0f} GB/s); "
        f"read probe over dy {adj['read_probe']['GB/s']:.0f} GB/s")
    pr, pc = workloads.pixel_sample(N0, N1, 256, 57)
    dx_s = dx[0].cpu().numpy()[pr, pc]
    dy_np = y[0].cpu().numpy() if not args.no_cpu_baseline else None
    del y
    cpu, err = None, None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.get()
        xd = x_np.astype(np.complex128)
        ref = orc.swdft2d(xd, n0, n1, windows=(q0, q1))
        err = rel(got, ref)
        dense["rel_err"] = rel(got_d, ref)
        dense["max_abs_err"] = float(np.max(np.abs(got_d - ref)))
        cpu = oracle_rate(orc, xd, n0, n1, P0, P1, args.cpu_seconds, 3003)
        adj_ref = orc.swdft2d_adjoint(dy_np.astype(np.complex128), N0, N1, pixels=(pr, pc))
        adj["rel_err"] = rel(dx_s, adj_ref)
    out = base_record(args, coeffs / step_s, step_s * 1e3, "f32", {
        "workload": "cplx2048: one 2048x512 complex64 image (re, im N(0,1)), 32x8 windows -> "
                    "2017x505x256 complex64 coefficients",
        "N0": N0, "N1": N1, "n0": n0, "n1": n1, "batch": 1, "algo": "tree",
        "coeffs_per_step": coeffs})
    out.update({"roofline": rf, "rel_err": err, "dense": dense, "adjoint": adj,
                "cpu_baseline": cpu})
    return out


def run_mixed1024(args, swd, dev) -> dict:
    """Mixed-radix tree: 1024 x 1024 real FP32, 12 x 12 windows (levels of
    radix 2, 2, 3 per side), the FP64 direct form on the same GPU; 9 x 9,
    24 x 24 and 12 x 16 windows on the same image as extra lines."""
    import numpy as np
    import torch

    import workloads
    wl = workloads.mixed1024()
    x_np = wl["x"]
    N0, N1 = x_np.shape
    n0, n1 = wl["n0"], wl["n1"]
    P0, P1 = N0 - n0 + 1, N1 - n1 + 1
    x = torch.from_numpy(x_np).to(dev).unsqueeze(0)
    stream = torch.cuda.current_stream(dev)
    plan = swd.Plan(N0, N1, n0, n1, torch.float32, batch=1)
    coeffs = plan.output_elems()
    alg_bytes = plan.output_bytes() + x.numel() * 4
    log(plan.describe())
    y, avg_ms, step_s, med_ms = forward_leg(plan, x, args, stream)
    rf = roofline(alg_bytes, avg_ms, f"tree_mixed_kernel<{n0},{n1},real>", med_ms=med_ms)
    log(f"mixed tree {n0}x{n1}: {avg_ms * 1e3:.1f} us/launch, {rf['achieved']:.0f} GB/s")
    q0, q1 = workloads.window_sample(P0, P1, 4096, 2008)
    got = sampled(y[0], q0, q1)
    del y
    torch.cuda.empty_cache()
    comp = None
    if not args.no_comparator:
        pd = swd.Plan(N0, N1, n0, n1, torch.float64, batch=1, algo="direct_f64")
        xd = x.double()
        yd = torch.empty(pd.out_shape, dtype=pd.out_dtype, device=dev)
        pd.forward(xd, out=yd)
        torch.cuda.synchronize()
        steps = max(3, min(args.steps, 20))
        d_ms, d_wall, _ = time_launches(lambda: pd.forward(xd, out=yd), steps, stream)
        comp = {"algo": "direct_f64", "value": coeffs / (d_wall / steps), "unit": "coeffs/s",
                "avg_launch_ms": d_ms, "dtype": "f64", "tree_speedup": d_ms / avg_ms}
        log(f"direct_f64 {n0}x{n1}: {d_ms:.2f} ms/launch")
        del yd
        torch.cuda.empty_cache()
    extra = []
    for (m0, m1) in ((9, 9), (24, 24), (12, 16)):
        pe = swd.Plan(N0, N1, m0, m1, torch.float32, batch=1)
        _, e_ms, _, _ = forward_leg(pe, x, args, stream)
        eb = pe.output_bytes() + x.numel() * 4
        extra.append({"n0": m0, "n1": m1, "avg_launch_us": e_ms * 1e3,
                      "coeffs_per_s": pe.output_elems() / (e_ms * 1e-3),
                      "achieved_GBps": eb / (e_ms * 1e-3) / 1e9,
                      "frac": eb / (e_ms * 1e-3) / 1e9 / PEAK_HBM_GBS})
        log(f"mixed tree {m0}x{m1}: {e_ms * 1e3:.1f} us/launch")
        torch.cuda.empty_cache()
    cpu, err = None, None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.get()
        xd = x_np.astype(np.float64)
        err = rel(got, orc.swdft2d(xd, n0, n1, windows=(q0, q1)))
        cpu = oracle_rate(orc, xd, n0, n1, P0, P1, args.cpu_seconds, 3008)
    out = base_record(args, coeffs / step_s, step_s * 1e3, "f32", {
        "workload": "mixed1024: one 1024x1024 real FP32 image, N(0,1), 12x12 windows "
                    "(mixed-radix tree, levels of radix 2, 2, 3) -> 1013x1013x144 complex64 "
                    "coefficients",
        "N0": N0, "N1": N1, "n0": n0, "n1": n1, "batch": 1, "algo": "tree (mixed radix)",
        "coeffs_per_step": coeffs})
    out.update({"roofline": rf, "rel_err": err, "comparator": comp, "other_windows": extra,
                "cpu_baseline": cpu})
    return out


def oracle_rate3(orc, x3d, n, P, seconds: float, seed: int):
    """Time the 3D oracle on a seeded window sample sized to about `seconds`."""
    import workloads
    q = workloads.window_sample3(P, 64, seed)
    t0 = time.perf_counter()
    orc.swdft3d(x3d, *n, windows=q)
    per_win = (time.perf_counter() - t0) / q[0].size
    total = P[0] * P[1] * P[2]
    nwin = int(min(total, max(256, seconds / per_win)))
    s = workloads.window_sample3(P, nwin, seed + 1)
    t0 = time.perf_counter()
    orc.swdft3d(x3d, *n, windows=s)
    dt = time.perf_counter() - t0
    nk = n[0] * n[1] * n[2]
    return {"value": s[0].size * nk / dt, "unit": "coeffs/s", "cores": orc.num_threads(),
            "kind": "oracle",
            "sample": f"{s[0].size} of the {P[0]}x{P[1]}x{P[2]} windows (seeded, corners "
                      f"included), {s[0].size * nk} coefficients in {dt:.1f} s"}


def run_vol128(args, swd, dev) -> dict:
    import numpy as np
    import torch

    import workloads
    wl = workloads.vol128()
    x_np, n = wl["x"], wl["n"]
    N = x_np.shape
    P = tuple(N[i] - n[i] + 1 for i in range(3))
    x = torch.from_numpy(x_np).to(dev).unsqueeze(0)
    plan = swd.Plan3D(*N, *n)
    coeffs = plan.output_elems()
    alg_bytes = coeffs * 8 + x.numel() * 4
    stream = torch.cuda.current_stream(dev)
    log(plan.describe())
    y, avg_ms, step_s, med_ms = forward_leg(plan, x, args, stream)
    rf = roofline(alg_bytes, avg_ms, "tree3_fwd_kernel<8,8,8,real>", med_ms=med_ms)
    log(f"tree3d: {avg_ms * 1e3:.1f} us/launch, {rf['achieved']:.0f} GB/s")
    q = workloads.window_sample3(P, 256, 3006)
    got = y[0][tuple(torch.from_numpy(a).to(dev) for a in q)].cpu().numpy()
    probe_ms, _, _ = time_launches(lambda: swd.write_probe(y), max(3, args.steps // 10), stream)
    probe = {"GB/s": coeffs * 8 / (probe_ms * 1e-3) / 1e9, "bytes": coeffs * 8}
    probe["frac"] = probe["GB/s"] / PEAK_HBM_GBS
    del y
    cpu, err = None, None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.get()
        xd = x_np.astype(np.float64)
        err = rel(got, orc.swdft3d(xd, *n, windows=q))
        cpu = oracle_rate3(orc, xd, n, P, args.cpu_seconds, 3007)
    out = base_record(args, coeffs / step_s, step_s * 1e3, "f32", {
        "workload": "vol128: one 128x128x128 real FP32 volume, N(0,1), 8x8x8 windows (3D "
                    "extension) -> 121x121x121x512 complex64 coefficients",
        "N": list(N), "n": list(n), "batch": 1, "algo": "tree3d", "coeffs_per_step": coeffs})
    out.update({"roofline": rf, "rel_err": err, "write_probe": probe, "cpu_baseline": cpu})
    return out


def run_stream1024(args, swd, dev) -> dict:
    """sin1024's rows pushed through a 2D stream (the real-time order of
    Sec. 4.3): throughput with 64-row pushes, and the latency of 1-row pushes."""
    import numpy as np
    import torch

    import workloads
    wl = workloads.sin1024()
    x_np, n0, n1 = wl["x"], wl["n0"], wl["n1"]
    N0, N1 = x_np.shape
    P0, P1 = N0 - n0 + 1, N1 - n1 + 1
    x = torch.from_numpy(x_np).to(dev)
    stream = torch.cuda.current_stream(dev)
    s = swd.Stream2D(N1, n0, n1)
    y = torch.empty((P0, P1, n0, n1), dtype=torch.complex64, device=dev)
    chunk = 64
    h = s.handle
    from paper_1707_08213_amd import _lib

    def one_pass():
        _lib.check(_lib.lib.swdft2d_stream_reset(h, stream.cuda_stream), "swdft2d_stream_reset")
        out = 0
        for r in range(0, N0, chunk):
            rows = min(chunk, N0 - r)
            cnt = _lib.lib.swdft2d_stream_completes(h, rows)
            _lib.check(_lib.lib.swdft2d_stream_push(h, x[r].data_ptr(), rows,
                                                    y[out].data_ptr() if cnt else None,
                                                    stream.cuda_stream), "swdft2d_stream_push")
            out += cnt

    for _ in range(max(1, args.warmup // 5)):
        one_pass()
    torch.cuda.synchronize()
    passes = max(2, args.steps // 10)
    t0 = time.perf_counter()
    for _ in range(passes):
        one_pass()
    torch.cuda.synchronize()
    per_pass = (time.perf_counter() - t0) / passes
    coeffs = P0 * P1 * n0 * n1
    alg_bytes = coeffs * 8 + N0 * N1 * 4
    achieved = alg_bytes / per_pass / 1e9
    # latency of one-row pushes in steady state (each completes one window row)
    _lib.check(_lib.lib.swdft2d_stream_reset(h, stream.cuda_stream), "swdft2d_stream_reset")
    first = N0 // 2
    for r in range(0, first, chunk):
        rows = min(chunk, first - r)
        cnt = _lib.lib.swdft2d_stream_completes(h, rows)
        _lib.check(_lib.lib.swdft2d_stream_push(h, x[r].data_ptr(), rows,
                                                y[0].data_ptr() if cnt else None,
                                                stream.cuda_stream), "swdft2d_stream_push")
    torch.cuda.synchronize()
    lat = []
    for r in range(first, first + 64):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        _lib.check(_lib.lib.swdft2d_stream_push(h, x[r].data_ptr(), 1, y[0].data_ptr(),
                                                stream.cuda_stream), "swdft2d_stream_push")
        b.record(stream)
        b.synchronize()
        lat.append(a.elapsed_time(b) * 1e3)
    lat.sort()
    err = None
    if not args.no_cpu_baseline:
        import oracle
        one_pass()
        torch.cuda.synchronize()
        q0, q1 = workloads.window_sample(P0, P1, 1024, 2006)
        got = sampled(y, q0, q1)
        err = rel(got, oracle.get().swdft2d(x_np.astype(np.float64), n0, n1, windows=(q0, q1)))
    out = base_record(args, coeffs / per_pass, per_pass * 1e3, "f32", {
        "workload": "stream1024: the 1024 rows of sin1024 pushed through a 2D stream in 64-row "
                    "calls (16x16 windows, tree state resident between calls)",
        "N1": N1, "n0": n0, "n1": n1, "rows": N0, "rows_per_push": chunk, "algo": "stream",
        "coeffs_per_step": coeffs})
    out["steps"] = passes
    out.update({"roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                             "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                             "kernel": "tree_stream_kernel<16,16,real> (16 calls per pass)",
                             "algorithmic_bytes_per_launch": alg_bytes,
                             "avg_launch_us": per_pass * 1e6},
                "one_row_push_us": {"median": lat[len(lat) // 2], "min": lat[0],
                                    "max": lat[-1]},
                "rel_err": err, "cpu_baseline": None})
    return out


def run_grad256(args, swd, dev) -> dict:
    import numpy as np
    import torch

    import workloads
    wl = workloads.grad256()
    x_np, w_np = wl["x"], wl["w"]
    B, N0, N1 = x_np.shape
    n0, n1 = wl["n0"], wl["n1"]
    x = torch.from_numpy(x_np).to(dev)
    w = torch.from_numpy(w_np).to(dev)
    plan = swd.Plan(N0, N1, n0, n1, torch.float32, batch=B)
    coeffs = plan.output_elems()
    stream = torch.cuda.current_stream(dev)
    log(plan.describe())
    y, f_ms, f_step, f_med = forward_leg(plan, x, args, stream)
    dy = 2.0 * w * y
    dx = torch.empty_like(x)
    for _ in range(args.warmup):
        plan.backward(dy, out=dx)
    torch.cuda.synchronize()
    b_ms, b_wall, _ = time_launches(lambda: plan.backward(dy, out=dx), args.steps, stream)
    b_step = b_wall / args.steps
    rf_f = roofline(plan.output_bytes() + x.numel() * 4, f_ms, "tree_fwd_kernel<16,16,real>",
                    med_ms=f_med)
    rf_b = roofline(plan.output_bytes() + x.numel() * 4, b_ms,
                    "tree_adj_kernel<16,16,real> + reduce")
    rprobe = read_probe_leg(swd, dy, stream)
    log(f"fwd {f_ms * 1e3:.1f} us, bwd {b_ms * 1e3:.1f} us ({rf_b['achieved']:.0f} GB/s); "
        f"read probe over dy {rprobe['GB/s']:.0f} GB/s")
    r, c = workloads.pixel_sample(N0, N1, 256, 55)
    err = None
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.get()
        errs = []
        t_or, n_or = 0.0, 0
        for b in (0, B - 1):
            dyb = dy[b].cpu().numpy().astype(np.complex128)
            t0 = time.perf_counter()
            ref = orc.swdft2d_adjoint(dyb, N0, N1, pixels=(r, c)).real
            t_or += time.perf_counter() - t0
            n_or += r.size
            errs.append(rel(dx[b].cpu().numpy()[r, c], ref))
        err = max(errs)
        cpu = {"value": n_or / t_or, "unit": "dx pixels/s (adjoint)", "cores": orc.num_threads(),
               "kind": "oracle", "sample": f"{n_or} sampled pixels of 2 images"}
    out = base_record(args, coeffs / (f_step + b_step), (f_step + b_step) * 1e3, "f32", {
        "workload": "grad256: 16 real FP32 256x256 images, 16x16 windows, forward + adjoint of "
                    "L = sum w|A|^2 (Bernoulli(0.25) band mask)",
        "N0": N0, "N1": N1, "n0": n0, "n1": n1, "batch": B, "algo": "tree",
        "coeffs_per_step": coeffs})
    out.update({"forward_ms": f_step * 1e3, "backward_ms": b_step * 1e3, "roofline": rf_b,
                "roofline_forward": rf_f, "read_probe": rprobe, "rel_err": err,
                "cpu_baseline": cpu})
    return out


def read_probe_leg(swd, buf, stream) -> dict:
    """Time the library's read probe over buf (the adjoint's dy): the
    empirical HBM read ceiling at that byte count."""
    import torch
    sink = torch.zeros(1, dtype=torch.float32, device=buf.device)
    swd.read_probe(buf, sink)
    torch.cuda.synchronize()
    ms, _, _ = time_launches(lambda: swd.read_probe(buf, sink), 10, stream)
    nbytes = buf.numel() * buf.element_size()
    gbs = nbytes / (ms * 1e-3) / 1e9
    return {"GB/s": gbs, "frac": gbs / PEAK_HBM_GBS, "bytes": nbytes}


def run_uneven64(args, swd, dev) -> dict:
    import numpy as np
    import torch

    import workloads
    imgs = workloads.uneven64()
    shapes = [(im["x"].shape[0], im["x"].shape[1], im["n0"], im["n1"]) for im in imgs]
    plan = swd.BatchedPlan(shapes)
    x = plan.pack([torch.from_numpy(im["x"]) for im in imgs], device=dev)
    y = torch.empty(plan.y_numel, dtype=torch.complex64, device=dev)
    coeffs = plan.output_elems()
    alg_bytes = coeffs * 8 + x.numel() * 4
    stream = torch.cuda.current_stream(dev)
    log(f"untuned: {plan.describe()}")
    for _ in range(max(1, args.warmup // 2)):
        plan.forward(x, out=y)
    torch.cuda.synchronize()
    u_ms, u_wall, _ = time_launches(lambda: plan.forward(x, out=y), max(3, args.steps // 5), stream)
    t0 = time.perf_counter()
    plan.tune(x, out=y)
    tune_s = time.perf_counter() - t0
    log(f"tuned in {tune_s:.1f} s: {plan.describe()}")
    for _ in range(max(1, args.warmup // 2)):
        plan.forward(x, out=y)
    torch.cuda.synchronize()
    steps = max(3, args.steps // 5)
    avg_ms, wall, _ = time_launches(lambda: plan.forward(x, out=y), steps, stream)
    step_s = wall / steps
    rf = roofline(alg_bytes, avg_ms, "persistent per-shape kernels (one graph launch)")
    log(f"batched: {avg_ms:.2f} ms/launch ({rf['achieved']:.0f} GB/s), untuned {u_ms:.2f} ms")
    err, cpu = None, None
    if not args.no_cpu_baseline:
        import oracle
        orc = oracle.get()
        errs, t_or, n_or = [], 0.0, 0
        outs = plan.unpack(y)
        for i, (im, s) in enumerate(zip(imgs, shapes)):
            P0, P1 = s[0] - s[2] + 1, s[1] - s[3] + 1
            q0, q1 = workloads.window_sample(P0, P1, 32, 5000 + i)
            got = sampled(outs[i], q0, q1)
            t1 = time.perf_counter()
            ref = orc.swdft2d(im["x"].astype(np.float64), s[2], s[3], windows=(q0, q1))
            t_or += time.perf_counter() - t1
            n_or += q0.size * s[2] * s[3]
            errs.append(rel(got, ref))
        err = max(errs)
        cpu = {"value": n_or / t_or, "unit": "coeffs/s", "cores": orc.num_threads(),
               "kind": "oracle", "sample": f"32 windows per image, {n_or} coefficients"}
    del y
    out = base_record(args, coeffs / step_s, step_s * 1e3, "f32", {
        "workload": "uneven64: 64 real FP32 images, sides from {128,256,512,1024}, windows from "
                    "{8x8,16x16,32x32,8x32}, one graph launch of persistent per-shape kernels",
        "images": len(shapes), "batch": len(shapes), "algo": "batched", "coeffs_per_step": coeffs})
    out.update({"roofline": rf, "rel_err": err, "untuned_ms": u_ms, "tune_seconds": tune_s,
                "plan": plan.describe(), "cpu_baseline": cpu})
    return out


WORKLOADS = {"sin1024": run_sin1024, "cplx2048": run_cplx2048, "grad256": run_grad256,
             "vol128": run_vol128, "stream1024": run_stream1024,
             "uneven64": run_uneven64, "mixed1024": run_mixed1024}


FIG4_WINDOWS = (4, 8, 16, 32, 64)
# ops per coefficient (Table 1 over n0 n1 outputs per window): complex
# multiply-adds of Eq. (2), butterflies of a radix-2 2D FFT, node operations
# of the tree (Eq. (8))
FIG4_OPS = {"direct_f64": lambda n: n * n, "swfft": lambda n: (2 * (n.bit_length() - 1)) / 2,
            "tree": lambda n: 2 * (n * n - 1) / (n * n)}


def run_fig4(args, swd, dev) -> str:
    """Fig. 4 on the GPU: a seeded N(0,1) real array of 100 x 100 (the paper's
    size) and of 1024 x 1024, square windows n = 4..64, each through the FP64
    direct form of Eq. (2) (on the FP32 values widened exactly), the FP32
    per-window FFT and the FP32 tree. Times are averages of HIP event pairs
    around back-to-back launches; errors are normwise relative to the FP64
    direct output (to the per-window FFT where the direct form would take
    seconds per call)."""
    import numpy as np
    import torch

    import workloads
    stream = torch.cuda.current_stream(dev)
    lines = ["| N | n | algorithm | dtype | ops/coeff | us/call | coeffs/s | output GB/s | "
             "tree speedup | rel err |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    for N in (100, 1024):
        x32 = torch.from_numpy(workloads.normal_real((N, N), workloads.WORKLOAD_SEEDS["fig4"]))
        x32 = x32.to(dev)
        for n in FIG4_WINDOWS:
            P = N - n + 1
            coeffs = P * P * n * n
            res = {}
            ref = None
            for algo in ("direct_f64", "swfft", "tree"):
                est_s = coeffs * n * n / 4e12 if algo == "direct_f64" else 0.0
                if est_s > 1.0:
                    log(f"fig4 N={N} n={n} {algo}: skipped (about {est_s:.0f} s per call)")
                    continue
                x = (x32.double() if algo == "direct_f64" else x32).unsqueeze(0)
                plan = swd.Plan(N, N, n, n, dtype=x.dtype, batch=1, algo=algo)
                y = torch.empty(plan.out_shape, dtype=plan.out_dtype, device=dev)
                plan.forward(x, out=y)
                torch.cuda.synchronize()
                xp, yp, sp = x.data_ptr(), y.data_ptr(), stream.cuda_stream

                def call():
                    plan.exec_ptr(xp, yp, sp)
                one, _, _ = time_launches(call, 1, stream)
                steps = int(min(args.steps * 10, max(3, 0.5e3 / max(one, 1e-3))))
                for _ in range(min(args.warmup, steps)):
                    call()
                # one event pair around back-to-back launches: the queue stays
                # full, so small calls are timed on the device, not the host
                avg_ms = time_batch(call, steps, stream)
                err = None
                if ref is None:
                    ref = y  # the first algorithm run is the reference
                else:
                    d = (y.to(ref.dtype) - ref).abs().max() / ref.abs().max()
                    err = float(d)
                res[algo] = (avg_ms, err, plan.describe())
                log(f"fig4 N={N} n={n} {algo}: {avg_ms * 1e3:.1f} us/call over {steps} calls"
                    + (f", rel err {err:.2e}" if err is not None else ""))
                if y is not ref:
                    del y
            del ref
            torch.cuda.empty_cache()
            t_tree = res["tree"][0]
            for algo, (avg_ms, err, _) in res.items():
                dtype = "f64" if algo == "direct_f64" else "f32"
                ob = coeffs * (16 if algo == "direct_f64" else 8)
                lines.append(
                    f"| {N} | {n} | {algo} | {dtype} | {FIG4_OPS[algo](n):.3g} | "
                    f"{avg_ms * 1e3:.1f} | {coeffs / (avg_ms * 1e-3):.3e} | "
                    f"{ob / (avg_ms * 1e-3) / 1e9:.0f} | {avg_ms / t_tree:.2f} | "
                    f"{'reference' if err is None else f'{err:.1e}'} |")
    return "\n".join(lines)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="sin1024", choices=sorted(WORKLOADS) + ["all"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparator", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target CPU time of the oracle sample")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain device copy of the output's size (reference for "
                         "hardware byte counters)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="summarise two rocprofv3 --pmc databases and exit (no GPU needed)")
    ap.add_argument("--fig4", action="store_true",
                    help="run the Fig. 4 speed comparison (markdown table) instead")
    ap.add_argument("--trace-summary", metavar="TRACE_DB",
                    help="summarise a rocprofv3 --kernel-trace database and exit (no GPU needed)")
    ap.add_argument("--counter-summary", metavar="PMC_DB",
                    help="summarise any rocprofv3 --pmc database and exit (no GPU needed)")
    args = ap.parse_args()
    if args.counter_summary:
        print(counter_summary(args.counter_summary))
        return 0
    if args.trace_summary:
        print(trace_summary(args.trace_summary))
        return 0
    if args.pmc_summary:
        # copy size = output bytes of the sin1024 workload (1009*1009*256 complex64)
        print(pmc_summary(args.pmc_summary[0], args.pmc_summary[1], 1009 * 1009 * 256 * 8,
                          TRAFFIC_FILE))
        return 0
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the transform shards over window rows with no exchange between GPUs)",
              file=sys.stderr)
        return 2

    import torch

    import paper_1707_08213_amd as swd
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.fig4:
        print(run_fig4(args, swd, dev), flush=True)
        return 0
    names = sorted(WORKLOADS) if args.workload == "all" else [args.workload]
    if "sin1024" in names:
        names.remove("sin1024")
        names.insert(0, "sin1024")
    rc = 0
    for name in names:
        out = WORKLOADS[name](args, swd, dev)
        print(json.dumps(out), flush=True)
        torch.cuda.empty_cache()
        if out.get("rel_err") is not None and out["rel_err"] > 1e-5:
            log(f"{name}: accuracy gate failed: rel err {out['rel_err']:.3e} > 1e-5")
            rc = 1
    return rc


if __name__ == "__main__":
    sys.exit(main())
