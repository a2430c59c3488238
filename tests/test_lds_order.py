"""LDS ordering of the two-wave forward tree kernels (CPU: compiles to assembly).

Two waves share a strip: each writes half of a chunk's rows of row levels
(Eq. 5) to LDS and reads all of them in the column phase (Eq. 6), with a
barrier between the column phase of chunk c and the row phase of chunk c + 1.
In the slab's first chunk the priming steps may only keep their row value in
a ring for the next chunk, and the compiler may then sink that LDS read past
the barrier, where the other wave already overwrites the row: an intermittent
wrong result. This test compiles two-wave kernels whose first chunk is all
priming steps and checks that no stretch between two barriers holds an LDS
read followed by an LDS write.
"""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_08213_amd", "csrc")
PROBE = os.path.join(ROOT, "tests", "asm", "lds_order_probe.hip")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def reads_then_writes(asm: str, wave_pattern: str = r"ELi2EEEv"):
    """(kernel, segment) pairs where, between two s_barrier, a ds_read comes
    before a ds_write, in the kernels whose mangled name matches wave_pattern."""
    found = []
    name, body = None, []
    funcs = {}
    for ln in asm.splitlines():
        m = re.match(r"^(_Z\S+):", ln)
        if m:
            name = m.group(1)
            funcs[name] = []
            continue
        if name is not None:
            if "s_endpgm" in ln:
                name = None
                continue
            funcs[name].append(ln)
    for fn, lines in funcs.items():
        if not re.search(wave_pattern, fn):
            continue
        seg, segs = [], []
        for ln in lines:
            if "s_barrier" in ln:
                segs.append(seg)
                seg = []
            elif "ds_read" in ln:
                seg.append("R")
            elif "ds_write" in ln:
                seg.append("W")
        segs.append(seg)
        for i, s in enumerate(segs):
            t = "".join(s)
            if "R" in t and "W" in t[t.index("R"):]:
                found.append((fn, i))
    return found


def test_scanner_flags_a_sunk_read():
    """The check itself: a read after the barrier and before the next row
    phase's writes is flagged; reads of a chunk after the barrier that ends
    its row phase are not."""
    good = "\n".join([
        "_ZN5swdft4tree15tree_fwd_kernelILi8ELi1ELb1ELi2ELi2EEEv:  ; @x",
        "  ds_write_b64 v1, v[2:3]", "  s_barrier", "  ds_read_b64 v[2:3], v1",
        "  s_barrier", "  ds_write_b64 v1, v[2:3]", "  s_barrier", "  s_endpgm"])
    bad = good.replace("  ds_read_b64 v[2:3], v1\n  s_barrier\n  ds_write_b64 v1, v[2:3]",
                       "  s_barrier\n  ds_read_b64 v[2:3], v1\n  ds_write_b64 v1, v[2:3]")
    assert bad != good
    assert reads_then_writes(good) == []
    assert len(reads_then_writes(bad)) == 1


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc is not installed")
def test_two_wave_first_chunk_reads_precede_barrier(tmp_path):
    out = tmp_path / "probe.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "--cuda-device-only", "-S", PROBE, "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    asm = out.read_text()
    kernels = re.findall(r"^(_ZN5swdft4tree15tree_fwd_kernel\S+ELi2EEEv\S*):", asm, re.M)
    assert len(kernels) == 3, kernels
    assert reads_then_writes(asm) == []
