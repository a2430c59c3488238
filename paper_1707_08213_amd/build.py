"""Compile libswdft2d.so (the HIP kernels and the C ABI) for gfx950 in-tree.

Usage: python paper_1707_08213_amd/build.py [-v]   (run as a script: importing the
package would load the library this builds)
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import time
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIBRARY = os.path.join(PKG, "libswdft2d.so")
SOURCES = ["abi.hip", "abi_noalloc.hip", "abi3d.hip", "abi_stream.hip", "tree3d_fwd.hip", "tree_stream.hip",
           "batched_host.hip", "tune.hip",
           "tree_config.hip", "tree_fwd.hip",
           "write_probe.hip", "tree_adj.hip", "direct_f64.hip", "swfft_r.hip", "swfft_c.hip",
           "tree_mixed.hip", "tree_mixed_pow2_r.hip", "tree_mixed_pow2_c.hip",
           "dense_mfma.hip",
           "dense_mfma_r.hip", "dense_mfma_c.hip", "batched.hip", "batched_tree_r.hip",
           "batched_tree_c.hip", "batched_dense_r.hip", "batched_dense_c.hip"] + [
    f"tree_{kind}_n{n}_{t}.hip" for kind in ("fwd", "adj") for n in (1, 2, 4, 8, 16, 32)
    for t in ("r", "c")] + [f"tree_fwd_n64_{t}.hip" for t in ("r", "c")] + [
    f"tree_fwd_n{n0}_{t}_{n1}.hip" for n0 in (16, 32) for t in ("r", "c") for n1 in (16, 32, 64)] + [
    f"tree_fwd_n64_{t}_{n1}.hip" for t in ("r", "c") for n1 in (16, 32, 64)] + [
    f"tree3d_fwd_n{n0}_{t}.hip" for n0 in (2, 4, 8, 16) for t in ("r", "c")] + ["tree3d_adj.hip"] + [
    f"tree3d_adj_n{n0}_{t}.hip" for n0 in (2, 4, 8, 16) for t in ("r", "c")] + [
    f"tree_stream_n{n0}_{t}.hip" for n0 in (1, 2, 4, 8, 16, 32) for t in ("r", "c")] + [
    f"tree_mixed_n{n0}_{t}.hip" for n0 in (3, 6, 9, 12, 24) for t in ("r", "c")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _deps(dep_file: str):
    """Files a translation unit read when it was last compiled (from the
    compiler's -MMD output), or None when unknown."""
    try:
        text = open(dep_file).read()
    except OSError:
        return None
    text = text.replace("\\\n", " ")
    _, _, rest = text.partition(":")
    return [f for f in rest.split() if f]


def _up_to_date(src_path: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return False
    deps = _deps(obj[:-2] + ".d")
    if deps is None:
        return False
    t = os.path.getmtime(obj)
    for f in [src_path] + deps:
        if not os.path.exists(f) or os.path.getmtime(f) >= t:
            return False
    return True


def _compile(src: str, verbose: bool, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    src_path = os.path.join(CSRC, src)
    if incremental and _up_to_date(src_path, obj):
        return obj
    cmd = [HIPCC, *FLAGS, "-MMD", "-MF", obj[:-2] + ".d", "-c", src_path, "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose:
        print(f"{time.time() - t0:6.1f} s  {src}", flush=True)
        noisy = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if noisy:
            print("\n".join(noisy), flush=True)
    return obj


def build(verbose: bool = False, jobs: int = 8, incremental: bool = False) -> str:
    """Compile every source (or, with incremental=True, only those whose
    object is older than the source or a header it includes) and link
    libswdft2d.so."""
    os.makedirs(BUILD, exist_ok=True)
    # the largest window instantiations take longest: start them first
    def cost(src):
        if src.startswith("batched_"):
            return 100
        parts = src[:-4].split("_")
        n0 = max([int(t[1:]) for t in parts if t[:1] == "n" and t[1:].isdigit()] or [0])
        n1 = int(parts[-1]) if parts[-1].isdigit() else 0
        return n0 * (4 if n1 else 1) + n1
    order = sorted(SOURCES, key=lambda s: -cost(s))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, incremental), order))
    tmp = LIBRARY + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIBRARY)
    return LIBRARY


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
