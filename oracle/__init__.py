"""FP64 oracle for the 2D sliding-window DFT and its 3D extension (TEST
INFRASTRUCTURE).

Only ``tests/``, the smoke check and the bench's CPU-baseline leg may import
this package. The GPU library never does, and the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, FP64, the definition of
Eq. (2) of Sec. 4.1 evaluated window by window, its explicit adjoint, and the
3D definition that the trees of Sec. 4.4 reach). This
wrapper only marshals numpy arrays and compiles the C file with gcc when the
shared object is missing or older than its source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "oracle.c")
LIBRARY = os.path.join(_HERE, "liboracle.so")

_lock = threading.Lock()
_default = None


def compile_library(out_path: str = LIBRARY, mutation: int = 0, openmp: bool = True) -> str:
    """Compile oracle.c with gcc (no fast-math, FP contraction off)."""
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", SOURCE, "-o", out_path + ".tmp", "-lm"]
    if openmp:
        cmd.insert(1, "-fopenmp")
    if mutation:
        cmd.insert(1, f"-DORACLE_MUTATION={int(mutation)}")
    subprocess.run(cmd, check=True)
    os.replace(out_path + ".tmp", out_path)
    return out_path


def _stale(path: str) -> bool:
    return (not os.path.exists(path)) or os.path.getmtime(path) < os.path.getmtime(SOURCE)


def _as_f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


class Oracle:
    """ctypes view of one build of oracle.c."""

    def __init__(self, path: str = LIBRARY):
        self.path = path
        lib = ctypes.CDLL(path)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.oracle_swdft2d.argtypes = [vp, vp, i64, i64, i32, i32, i32, vp, vp, i64, vp, vp]
        lib.oracle_swdft2d.restype = ctypes.c_int
        lib.oracle_swdft2d_adjoint.argtypes = [vp, vp, i64, i64, i32, i32, i32, vp, vp, i64, vp, vp]
        lib.oracle_swdft2d_adjoint.restype = ctypes.c_int
        lib.oracle_swdft3d.argtypes = [vp, vp, i64, i64, i64, i32, i32, i32, i32, vp, vp, vp,
                                       i64, vp, vp]
        lib.oracle_swdft3d.restype = ctypes.c_int
        lib.oracle_swdft3d_adjoint.argtypes = [vp, vp, i64, i64, i64, i32, i32, i32, i32, vp, vp,
                                               vp, i64, vp, vp]
        lib.oracle_swdft3d_adjoint.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        self.lib = lib

    def num_threads(self) -> int:
        return int(self.lib.oracle_num_threads())

    def set_threads(self, n: int) -> None:
        """Threads of later OpenMP regions (timing only; results do not depend on it)."""
        self.lib.oracle_set_threads(int(n))

    def swdft2d(self, x, n0: int, n1: int, windows=None, norm: str = "none") -> np.ndarray:
        """Direct 2D SWDFT of one N0 x N1 image (real or complex).

        windows: None for every window -> complex128 [P0, P1, n0, n1];
                 or (q0, q1) int arrays -> complex128 [len(q0), n0, n1].
        """
        x = np.asarray(x)
        if x.ndim != 2:
            raise ValueError("oracle.swdft2d takes one 2D image")
        N0, N1 = x.shape
        xr = _as_f64(x.real)
        xi = _as_f64(x.imag) if np.iscomplexobj(x) else None
        P0, P1 = N0 - n0 + 1, N1 - n1 + 1
        if windows is None:
            q0 = q1 = None
            nwin = P0 * P1
        else:
            q0 = np.ascontiguousarray(windows[0], dtype=np.int64)
            q1 = np.ascontiguousarray(windows[1], dtype=np.int64)
            nwin = q0.size
        yr = np.empty((nwin, n0, n1), np.float64)
        yi = np.empty((nwin, n0, n1), np.float64)
        rc = self.lib.oracle_swdft2d(_ptr(xr), _ptr(xi), N0, N1, n0, n1, int(norm == "ortho"),
                                     _ptr(q0), _ptr(q1), nwin, _ptr(yr), _ptr(yi))
        if rc != 0:
            raise ValueError(f"oracle_swdft2d rejected N=({N0},{N1}) n=({n0},{n1})")
        y = yr + 1j * yi
        return y.reshape(P0, P1, n0, n1) if windows is None else y

    def swdft2d_adjoint(self, dy, N0: int, N1: int, pixels=None, norm: str = "none") -> np.ndarray:
        """Explicit adjoint: dy complex [P0, P1, n0, n1] -> dx complex.

        pixels: None -> [N0, N1]; or (r, c) int arrays -> [len(r)].
        """
        dy = np.asarray(dy)
        P0, P1, n0, n1 = dy.shape
        if P0 != N0 - n0 + 1 or P1 != N1 - n1 + 1:
            raise ValueError("dy shape does not match (N0, N1)")
        gr = _as_f64(dy.real)
        gi = _as_f64(dy.imag)
        if pixels is None:
            r = c = None
            npix = N0 * N1
        else:
            r = np.ascontiguousarray(pixels[0], dtype=np.int64)
            c = np.ascontiguousarray(pixels[1], dtype=np.int64)
            npix = r.size
        dxr = np.empty(npix, np.float64)
        dxi = np.empty(npix, np.float64)
        rc = self.lib.oracle_swdft2d_adjoint(_ptr(gr), _ptr(gi), N0, N1, n0, n1,
                                             int(norm == "ortho"), _ptr(r), _ptr(c), npix,
                                             _ptr(dxr), _ptr(dxi))
        if rc != 0:
            raise ValueError("oracle_swdft2d_adjoint rejected its arguments")
        dx = dxr + 1j * dxi
        return dx.reshape(N0, N1) if pixels is None else dx


    def swdft3d(self, x, n0: int, n1: int, n2: int, windows=None, norm: str = "none") -> np.ndarray:
        """Direct 3D SWDFT of one N0 x N1 x N2 volume (real or complex).

        windows: None for every window -> complex128 [P0, P1, P2, n0, n1, n2];
                 or (q0, q1, q2) int arrays -> complex128 [len(q0), n0, n1, n2].
        """
        x = np.asarray(x)
        if x.ndim != 3:
            raise ValueError("oracle.swdft3d takes one 3D volume")
        N0, N1, N2 = x.shape
        xr = _as_f64(x.real)
        xi = _as_f64(x.imag) if np.iscomplexobj(x) else None
        P0, P1, P2 = N0 - n0 + 1, N1 - n1 + 1, N2 - n2 + 1
        if windows is None:
            q0 = q1 = q2 = None
            nwin = P0 * P1 * P2
        else:
            q0, q1, q2 = (np.ascontiguousarray(w, dtype=np.int64) for w in windows)
            nwin = q0.size
        yr = np.empty((nwin, n0, n1, n2), np.float64)
        yi = np.empty((nwin, n0, n1, n2), np.float64)
        rc = self.lib.oracle_swdft3d(_ptr(xr), _ptr(xi), N0, N1, N2, n0, n1, n2,
                                     int(norm == "ortho"), _ptr(q0), _ptr(q1), _ptr(q2), nwin,
                                     _ptr(yr), _ptr(yi))
        if rc != 0:
            raise ValueError(f"oracle_swdft3d rejected N=({N0},{N1},{N2}) n=({n0},{n1},{n2})")
        y = yr + 1j * yi
        return y.reshape(P0, P1, P2, n0, n1, n2) if windows is None else y

    def swdft3d_adjoint(self, dy, N0: int, N1: int, N2: int, voxels=None,
                        norm: str = "none") -> np.ndarray:
        """Explicit 3D adjoint: dy complex [P0, P1, P2, n0, n1, n2] -> dx complex.

        voxels: None -> [N0, N1, N2]; or (r0, r1, r2) int arrays -> [len(r0)].
        """
        dy = np.asarray(dy)
        P0, P1, P2, n0, n1, n2 = dy.shape
        if (P0, P1, P2) != (N0 - n0 + 1, N1 - n1 + 1, N2 - n2 + 1):
            raise ValueError("dy shape does not match (N0, N1, N2)")
        gr = _as_f64(dy.real)
        gi = _as_f64(dy.imag)
        if voxels is None:
            v0 = v1 = v2 = None
            nvox = N0 * N1 * N2
        else:
            v0, v1, v2 = (np.ascontiguousarray(v, dtype=np.int64) for v in voxels)
            nvox = v0.size
        dxr = np.empty(nvox, np.float64)
        dxi = np.empty(nvox, np.float64)
        rc = self.lib.oracle_swdft3d_adjoint(_ptr(gr), _ptr(gi), N0, N1, N2, n0, n1, n2,
                                             int(norm == "ortho"), _ptr(v0), _ptr(v1), _ptr(v2),
                                             nvox, _ptr(dxr), _ptr(dxi))
        if rc != 0:
            raise ValueError("oracle_swdft3d_adjoint rejected its arguments")
        dx = dxr + 1j * dxi
        return dx.reshape(N0, N1, N2) if voxels is None else dx


def get() -> Oracle:
    """The default (unmutated) oracle, compiled on first use if needed."""
    global _default
    with _lock:
        if _default is None:
            if _stale(LIBRARY):
                compile_library(LIBRARY)
            _default = Oracle(LIBRARY)
        return _default


def swdft2d(x, n0, n1, windows=None, norm="none"):
    return get().swdft2d(x, n0, n1, windows=windows, norm=norm)


def swdft2d_adjoint(dy, N0, N1, pixels=None, norm="none"):
    return get().swdft2d_adjoint(dy, N0, N1, pixels=pixels, norm=norm)


def swdft3d(x, n0, n1, n2, windows=None, norm="none"):
    return get().swdft3d(x, n0, n1, n2, windows=windows, norm=norm)


def swdft3d_adjoint(dy, N0, N1, N2, voxels=None, norm="none"):
    return get().swdft3d_adjoint(dy, N0, N1, N2, voxels=voxels, norm=norm)
