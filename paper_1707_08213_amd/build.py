"""Compile libswdft2d.so (the HIP kernels and the C ABI) for gfx950 in-tree.

Usage: python paper_1707_08213_amd/build.py [-v]   (run as a script: importing the
package would load the library this builds)
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIBRARY = os.path.join(PKG, "libswdft2d.so")
SOURCES = ["abi.hip", "batched_host.hip", "tune.hip", "tree_config.hip", "tree_fwd.hip",
           "write_probe.hip", "tree_adj.hip", "direct_f64.hip", "dense_mfma.hip",
           "dense_mfma_r.hip", "dense_mfma_c.hip", "batched.hip", "batched_tree_r.hip",
           "batched_tree_c.hip", "batched_dense_r.hip", "batched_dense_c.hip"] + [
    f"tree_{kind}_n{n}_{t}.hip" for kind in ("fwd", "adj") for n in (1, 2, 4, 8, 16, 32)
    for t in ("r", "c")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _newest_header() -> float:
    newest = 0.0
    for d in (CSRC, os.path.join(ROOT, "include")):
        for f in os.listdir(d):
            if f.endswith(".h"):
                newest = max(newest, os.path.getmtime(os.path.join(d, f)))
    return newest


def _compile(src: str, verbose: bool, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t > os.path.getmtime(os.path.join(CSRC, src)) and t > _newest_header():
            return obj
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    noisy = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if verbose and noisy:
        print("\n".join(noisy), flush=True)
    return obj


def build(verbose: bool = False, jobs: int = 8, incremental: bool = False) -> str:
    """Compile every source (or, with incremental=True, only those older than
    their source or any header) and link libswdft2d.so."""
    os.makedirs(BUILD, exist_ok=True)
    # the largest window instantiations take longest: start them first
    def cost(src):
        if src.startswith("batched_"):
            return 100
        return max([int(t[1:]) for t in src[:-4].split("_") if t[:1] == "n" and t[1:].isdigit()]
                   or [0])
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
