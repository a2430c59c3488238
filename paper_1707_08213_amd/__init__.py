"""MI355X-native 2D Tree Sliding-Window DFT (Richardson & Eddy, arXiv 1707.08213).

Python face of libswdft2d.so. PyTorch supplies device memory and the stream;
every arithmetic step runs in the library's HIP kernels, called through the C
ABI of include/swdft2d.h (see ``_lib``).

    y = swdft2d(x, n0, n1)              # x: [B,] N0 x N1 on cuda, float32/complex64
    y.shape == (B, P0, P1, n0, n1)      # P_i = N_i - n_i + 1, complex64

``SWDFT2dFn`` wraps forward and the hand-written adjoint as an autograd
function.
"""
from __future__ import annotations

import ctypes
import threading

import torch

from . import _lib
from ._lib import SwdftError, check, lib

__all__ = ["Plan", "BatchedPlan", "Plan3D", "Stream2D", "swdft2d", "swdft2d_batched",
           "swdft2d_backward", "swdft3d", "SWDFT2dFn", "write_probe", "read_probe", "SwdftError", "output_shape"]

_DTYPES = {
    torch.float32: _lib.SWDFT_R32, torch.complex64: _lib.SWDFT_C32,
    torch.float64: _lib.SWDFT_R64, torch.complex128: _lib.SWDFT_C64,
}
_OUT_DTYPE = {_lib.SWDFT_R32: torch.complex64, _lib.SWDFT_C32: torch.complex64,
              _lib.SWDFT_R64: torch.complex128, _lib.SWDFT_C64: torch.complex128}
_NORMS = {"none": _lib.SWDFT_NORM_NONE, "ortho": _lib.SWDFT_NORM_ORTHO}
_ALGOS = {"auto": _lib.SWDFT_ALGO_AUTO, "tree": _lib.SWDFT_ALGO_TREE,
          "dense_bf16x2": _lib.SWDFT_ALGO_DENSE_BF16X2, "direct_f64": _lib.SWDFT_ALGO_DIRECT_F64,
          "swfft": _lib.SWDFT_ALGO_SWFFT}


def output_shape(N0: int, N1: int, n0: int, n1: int, batch: int = 1):
    return (batch, N0 - n0 + 1, N1 - n1 + 1, n0, n1)


class Plan:
    """One swdft2d plan: `batch` images of N0 x N1, n0 x n1 windows."""

    def __init__(self, N0, N1, n0, n1, dtype=torch.float32, batch=1, norm="none", algo="auto"):
        if dtype not in _DTYPES:
            raise TypeError(f"unsupported dtype {dtype}")
        self.N0, self.N1, self.n0, self.n1, self.batch = int(N0), int(N1), int(n0), int(n1), int(batch)
        self.dtype = dtype
        self.code = _DTYPES[dtype]
        h = ctypes.c_void_p()
        check(lib.swdft2d_plan(ctypes.byref(h), self.N0, self.N1, self.n0, self.n1, self.code,
                               self.batch), "swdft2d_plan")
        self.handle = h
        try:
            check(lib.swdft2d_set_norm(h, _NORMS[norm]), "swdft2d_set_norm")
            check(lib.swdft2d_set_algo(h, _ALGOS[algo]), "swdft2d_set_algo")
        except Exception:
            lib.swdft2d_destroy(h)
            self.handle = None
            raise
        self.norm, self.algo = norm, algo

    @property
    def out_shape(self):
        return output_shape(self.N0, self.N1, self.n0, self.n1, self.batch)

    @property
    def out_dtype(self):
        return _OUT_DTYPE[self.code]

    def output_elems(self) -> int:
        return int(lib.swdft2d_output_elems(self.handle))

    def output_bytes(self) -> int:
        return int(lib.swdft2d_output_bytes(self.handle))

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(512)
        check(lib.swdft2d_describe(self.handle, buf, 512), "swdft2d_describe")
        return buf.value.decode()

    # raw-pointer entry points (device addresses as ints)
    def exec_ptr(self, x_ptr: int, y_ptr: int, stream: int = 0) -> None:
        check(lib.swdft2d_exec(self.handle, x_ptr, y_ptr, stream), "swdft2d_exec")

    def backward_ptr(self, dy_ptr: int, dx_ptr: int, stream: int = 0) -> None:
        check(lib.swdft2d_backward(self.handle, dy_ptr, dx_ptr, stream), "swdft2d_backward")

    # tensor entry points
    def _check_x(self, x: torch.Tensor):
        want = (self.batch, self.N0, self.N1)
        if x.dtype != self.dtype or not x.is_cuda or not x.is_contiguous() or \
                tuple(x.shape) != want:
            raise ValueError(f"x must be a contiguous cuda {self.dtype} tensor of shape {want}, "
                             f"got {x.dtype} {tuple(x.shape)} on {x.device}")

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check_x(x)
        if out is None:
            out = torch.empty(self.out_shape, dtype=self.out_dtype, device=x.device)
        elif (out.dtype != self.out_dtype or tuple(out.shape) != self.out_shape
              or not out.is_contiguous() or out.device != x.device):
            raise ValueError("out has the wrong shape, dtype or device")
        with torch.cuda.device(x.device):
            stream = torch.cuda.current_stream(x.device).cuda_stream
            self.exec_ptr(x.data_ptr(), out.data_ptr(), stream)
        return out

    def backward(self, dy: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if dy.dtype != self.out_dtype or tuple(dy.shape) != self.out_shape or \
                not dy.is_contiguous() or not dy.is_cuda:
            raise ValueError(f"dy must be a contiguous cuda {self.out_dtype} tensor of shape "
                             f"{self.out_shape}")
        if out is None:
            out = torch.empty((self.batch, self.N0, self.N1), dtype=self.dtype, device=dy.device)
        with torch.cuda.device(dy.device):
            stream = torch.cuda.current_stream(dy.device).cuda_stream
            self.backward_ptr(dy.data_ptr(), out.data_ptr(), stream)
        return out

    def tune(self, x: torch.Tensor, out: torch.Tensor | None = None) -> None:
        """Time candidate tile shapes / algorithms on x and keep the fastest
        (overwrites `out`; blocks until done)."""
        self._check_x(x)
        if out is None:
            out = torch.empty(self.out_shape, dtype=self.out_dtype, device=x.device)
        with torch.cuda.device(x.device):
            stream = torch.cuda.current_stream(x.device).cuda_stream
            check(lib.swdft2d_tune(self.handle, x.data_ptr(), out.data_ptr(), stream),
                  "swdft2d_tune")

    def close(self):
        if getattr(self, "handle", None) is not None:
            check(lib.swdft2d_destroy(self.handle), "swdft2d_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedPlan:
    """Many images of uneven sizes and window shapes in one exec.

    shapes: list of (N0, N1, n0, n1) with n0, n1 in {8, 16, 32}. Inputs are
    packed into one flat tensor (image i at x_offsets[i], row-major) and so
    are outputs (image i's [P0, P1, n0, n1] block at y_offsets[i])."""

    def __init__(self, shapes, dtype=torch.float32, norm="none", algo="auto"):
        if dtype not in (torch.float32, torch.complex64):
            raise TypeError("batched plans take float32 or complex64 input")
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.dtype = dtype
        self.code = _DTYPES[dtype]
        self.x_offsets, self.y_offsets, self.out_shapes = [], [], []
        xo = yo = 0
        descs = (_lib.Desc * len(self.shapes))()
        for i, (N0, N1, n0, n1) in enumerate(self.shapes):
            P0, P1 = N0 - n0 + 1, N1 - n1 + 1
            descs[i] = _lib.Desc(N0, N1, n0, n1, xo, yo)
            self.x_offsets.append(xo)
            self.y_offsets.append(yo)
            self.out_shapes.append((P0, P1, n0, n1))
            xo += N0 * N1
            yo += max(P0, 0) * max(P1, 0) * n0 * n1
        self.x_numel, self.y_numel = xo, yo
        h = ctypes.c_void_p()
        check(lib.swdft2d_plan_batched(ctypes.byref(h), ctypes.cast(descs, ctypes.c_void_p),
                                       len(self.shapes), self.code), "swdft2d_plan_batched")
        self.handle = h
        try:
            check(lib.swdft2d_set_norm(h, _NORMS[norm]), "swdft2d_set_norm")
            check(lib.swdft2d_set_algo(h, _ALGOS[algo]), "swdft2d_set_algo")
        except Exception:
            lib.swdft2d_destroy(h)
            self.handle = None
            raise

    def pack(self, images, device=None) -> torch.Tensor:
        """Concatenate images (each [N0, N1]) into the packed input layout."""
        flat = [im.reshape(-1) for im in images]
        x = torch.cat(flat).to(device=device if device is not None else flat[0].device)
        return x.to(self.dtype).contiguous()

    def unpack(self, y: torch.Tensor):
        """Views of the packed output, one [P0, P1, n0, n1] tensor per image."""
        out = []
        for off, shp in zip(self.y_offsets, self.out_shapes):
            n = shp[0] * shp[1] * shp[2] * shp[3]
            out.append(y[off:off + n].view(shp))
        return out

    def output_elems(self) -> int:
        return int(lib.swdft2d_output_elems(self.handle))

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(4096)
        check(lib.swdft2d_describe(self.handle, buf, 4096), "swdft2d_describe")
        return buf.value.decode()

    def _check(self, x, out):
        if x.dtype != self.dtype or not x.is_cuda or not x.is_contiguous() or x.numel() != self.x_numel:
            raise ValueError(f"x must be a contiguous cuda {self.dtype} tensor of {self.x_numel} elements")
        if out is None:
            out = torch.empty(self.y_numel, dtype=torch.complex64, device=x.device)
        elif out.dtype != torch.complex64 or out.numel() != self.y_numel or not out.is_contiguous():
            raise ValueError("out has the wrong size or dtype")
        return out

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self._check(x, out)
        with torch.cuda.device(x.device):
            stream = torch.cuda.current_stream(x.device).cuda_stream
            check(lib.swdft2d_exec(self.handle, x.data_ptr(), out.data_ptr(), stream),
                  "swdft2d_exec")
        return out

    def tune(self, x: torch.Tensor, out: torch.Tensor | None = None) -> None:
        out = self._check(x, out)
        with torch.cuda.device(x.device):
            stream = torch.cuda.current_stream(x.device).cuda_stream
            check(lib.swdft2d_tune(self.handle, x.data_ptr(), out.data_ptr(), stream),
                  "swdft2d_tune")

    def close(self):
        if getattr(self, "handle", None) is not None:
            check(lib.swdft2d_destroy(self.handle), "swdft2d_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def swdft2d_batched(images, windows, norm: str = "none", algo: str = "auto"):
    """Transform a list of 2D images (float32 or complex64, on one cuda device)
    with per-image windows [(n0, n1), ...] in one exec; returns a list of
    [P0, P1, n0, n1] complex64 tensors (views of one packed buffer)."""
    shapes = [(im.shape[0], im.shape[1], w[0], w[1]) for im, w in zip(images, windows)]
    plan = BatchedPlan(shapes, dtype=images[0].dtype, norm=norm, algo=algo)
    y = plan.forward(plan.pack(images))
    return plan.unpack(y)


_cache_lock = threading.Lock()
_plan_cache: dict = {}


def _cached_plan(N0, N1, n0, n1, dtype, batch, norm, algo) -> Plan:
    # A plan holds one adjoint workspace and its calls must not overlap, so
    # plans are cached per host thread and per device stream: calls on one
    # (thread, stream) pair are ordered by that stream.
    stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
    key = (N0, N1, n0, n1, dtype, batch, norm, algo, threading.get_ident(),
           torch.cuda.current_device() if torch.cuda.is_available() else -1, stream)
    with _cache_lock:
        p = _plan_cache.get(key)
        if p is None:
            p = Plan(N0, N1, n0, n1, dtype=dtype, batch=batch, norm=norm, algo=algo)
            _plan_cache[key] = p
        return p


def _batched(x: torch.Tensor):
    if x.dim() == 2:
        return x.unsqueeze(0), True
    if x.dim() == 3:
        return x, False
    raise ValueError("x must be [N0, N1] or [B, N0, N1]")


def swdft2d(x: torch.Tensor, n0: int, n1: int, norm: str = "none", algo: str = "auto") -> torch.Tensor:
    """2D sliding-window DFT of every n0 x n1 window of x ([N0,N1] or [B,N0,N1])."""
    xb, squeeze = _batched(x.contiguous())
    B, N0, N1 = xb.shape
    y = _cached_plan(N0, N1, n0, n1, xb.dtype, B, norm, algo).forward(xb)
    return y[0] if squeeze else y


class Plan3D:
    """One swdft3d plan: `batch` volumes of N0 x N1 x N2, n0 x n1 x n2 windows
    (the 3D extension of Sec. 4.4)."""

    def __init__(self, N0, N1, N2, n0, n1, n2, dtype=torch.float32, batch=1, norm="none"):
        if dtype not in (torch.float32, torch.complex64):
            raise TypeError(f"3D plans take float32 or complex64 input, got {dtype}")
        self.N = (int(N0), int(N1), int(N2))
        self.n = (int(n0), int(n1), int(n2))
        self.batch, self.dtype = int(batch), dtype
        h = ctypes.c_void_p()
        check(lib.swdft3d_plan(ctypes.byref(h), *self.N, *self.n, _DTYPES[dtype], self.batch),
              "swdft3d_plan")
        self.handle = h
        try:
            check(lib.swdft3d_set_norm(h, _NORMS[norm]), "swdft3d_set_norm")
        except Exception:
            lib.swdft3d_destroy(h)
            self.handle = None
            raise
        self.norm = norm

    @property
    def out_shape(self):
        P = tuple(self.N[i] - self.n[i] + 1 for i in range(3))
        return (self.batch,) + P + self.n

    @property
    def out_dtype(self):
        return torch.complex64

    def output_elems(self) -> int:
        return int(lib.swdft3d_output_elems(self.handle))

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(512)
        check(lib.swdft3d_describe(self.handle, buf, 512), "swdft3d_describe")
        return buf.value.decode()

    def exec_ptr(self, x_ptr: int, y_ptr: int, stream: int = 0) -> None:
        check(lib.swdft3d_exec(self.handle, x_ptr, y_ptr, stream), "swdft3d_exec")

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        want = (self.batch,) + self.N
        if x.dtype != self.dtype or not x.is_cuda or not x.is_contiguous() or \
                tuple(x.shape) != want:
            raise ValueError(f"x must be a contiguous cuda {self.dtype} tensor of shape {want}, "
                             f"got {x.dtype} {tuple(x.shape)} on {x.device}")
        if out is None:
            out = torch.empty(self.out_shape, dtype=torch.complex64, device=x.device)
        elif (out.dtype != torch.complex64 or tuple(out.shape) != self.out_shape
              or not out.is_contiguous() or out.device != x.device):
            raise ValueError("out has the wrong shape, dtype or device")
        with torch.cuda.device(x.device):
            stream = torch.cuda.current_stream(x.device).cuda_stream
            self.exec_ptr(x.data_ptr(), out.data_ptr(), stream)
        return out

    def backward(self, dy: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Adjoint: dy [B,P0,P1,P2,n0,n1,n2] complex64 -> dx [B,N0,N1,N2] (x's dtype)."""
        if dy.dtype != torch.complex64 or tuple(dy.shape) != self.out_shape or \
                not dy.is_contiguous() or not dy.is_cuda:
            raise ValueError(f"dy must be a contiguous cuda complex64 tensor of shape "
                             f"{self.out_shape}")
        want = (self.batch,) + self.N
        if out is None:
            out = torch.empty(want, dtype=self.dtype, device=dy.device)
        elif (out.dtype != self.dtype or tuple(out.shape) != want or not out.is_contiguous()
              or out.device != dy.device):
            raise ValueError("out has the wrong shape, dtype or device")
        with torch.cuda.device(dy.device):
            stream = torch.cuda.current_stream(dy.device).cuda_stream
            check(lib.swdft3d_backward(self.handle, dy.data_ptr(), out.data_ptr(), stream),
                  "swdft3d_backward")
        return out

    def close(self):
        if getattr(self, "handle", None) is not None:
            check(lib.swdft3d_destroy(self.handle), "swdft3d_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream2D:
    """Streaming 2D SWDFT over rows of length N1 (the real-time order of
    Sec. 4.3): push(rows) returns the window rows those rows complete."""

    def __init__(self, N1, n0, n1, dtype=torch.float32, norm="none"):
        if dtype not in (torch.float32, torch.complex64):
            raise TypeError(f"streams take float32 or complex64 input, got {dtype}")
        self.N1, self.n0, self.n1, self.dtype = int(N1), int(n0), int(n1), dtype
        h = ctypes.c_void_p()
        check(lib.swdft2d_stream_create(ctypes.byref(h), self.N1, self.n0, self.n1, _DTYPES[dtype]),
              "swdft2d_stream_create")
        self.handle = h
        try:
            check(lib.swdft2d_stream_set_norm(h, _NORMS[norm]), "swdft2d_stream_set_norm")
        except Exception:
            lib.swdft2d_stream_destroy(h)
            self.handle = None
            raise

    @property
    def rows(self) -> int:
        return int(lib.swdft2d_stream_rows(self.handle))

    def push(self, x: torch.Tensor) -> torch.Tensor:
        """x: contiguous cuda [R, N1] rows -> complex64 [count, P1, n0, n1]."""
        if x.dtype != self.dtype or not x.is_cuda or not x.is_contiguous() or \
                x.dim() != 2 or x.shape[1] != self.N1:
            raise ValueError(f"x must be a contiguous cuda {self.dtype} tensor [R, {self.N1}]")
        count = int(lib.swdft2d_stream_completes(self.handle, x.shape[0]))
        P1 = self.N1 - self.n1 + 1
        y = torch.empty((count, P1, self.n0, self.n1), dtype=torch.complex64, device=x.device)
        with torch.cuda.device(x.device):
            stream = torch.cuda.current_stream(x.device).cuda_stream
            check(lib.swdft2d_stream_push(self.handle, x.data_ptr(), x.shape[0],
                                          y.data_ptr() if count else None, stream),
                  "swdft2d_stream_push")
        return y

    def reset(self) -> None:
        stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else None
        check(lib.swdft2d_stream_reset(self.handle, stream), "swdft2d_stream_reset")

    def close(self):
        if getattr(self, "handle", None) is not None:
            check(lib.swdft2d_stream_destroy(self.handle), "swdft2d_stream_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def swdft3d(x: torch.Tensor, n0: int, n1: int, n2: int, norm: str = "none") -> torch.Tensor:
    """3D sliding-window DFT of every n0 x n1 x n2 window of x ([N0,N1,N2] or
    [B,N0,N1,N2]) -> complex64 [B,P0,P1,P2,n0,n1,n2]."""
    x = x.contiguous()
    squeeze = x.dim() == 3
    xb = x.unsqueeze(0) if squeeze else x
    B, N0, N1, N2 = xb.shape
    y = _cached_plan3d(N0, N1, N2, n0, n1, n2, xb.dtype, B, norm).forward(xb)
    return y[0] if squeeze else y


def _cached_plan3d(N0, N1, N2, n0, n1, n2, dtype, batch, norm) -> Plan3D:
    # per host thread and device stream, like _cached_plan (a plan holds one
    # adjoint workspace)
    stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
    key = ("3d", N0, N1, N2, n0, n1, n2, dtype, batch, norm, threading.get_ident(),
           torch.cuda.current_device() if torch.cuda.is_available() else -1, stream)
    with _cache_lock:
        p = _plan_cache.get(key)
        if p is None:
            p = Plan3D(N0, N1, N2, n0, n1, n2, dtype=dtype, batch=batch, norm=norm)
            _plan_cache[key] = p
        return p


def swdft3d_backward(dy: torch.Tensor, N0: int, N1: int, N2: int, dtype=torch.float32,
                     norm: str = "none") -> torch.Tensor:
    """3D adjoint: dy [B,P0,P1,P2,n0,n1,n2] -> dx [B,N0,N1,N2] (Re of M^H dy for
    real dtypes)."""
    squeeze = dy.dim() == 6
    dyb = dy.unsqueeze(0) if squeeze else dy
    B, n0, n1, n2 = dyb.shape[0], dyb.shape[4], dyb.shape[5], dyb.shape[6]
    dx = _cached_plan3d(N0, N1, N2, n0, n1, n2, dtype, B, norm).backward(dyb.contiguous())
    return dx[0] if squeeze else dx


class SWDFT3dFn(torch.autograd.Function):
    """y = swdft3d(x); the backward pass runs the library's 3D adjoint kernel
    (Re(M^H gy) for real x, PyTorch's conjugate-Wirtinger convention)."""

    @staticmethod
    def forward(ctx, x, n0, n1, n2, norm="none"):
        ctx.meta = (x.shape, x.dtype, n0, n1, n2, norm)
        return swdft3d(x, n0, n1, n2, norm=norm)

    @staticmethod
    def backward(ctx, gy):
        shape, dtype, n0, n1, n2, norm = ctx.meta
        N0, N1, N2 = shape[-3], shape[-2], shape[-1]
        dx = swdft3d_backward(gy.contiguous(), N0, N1, N2, dtype=dtype, norm=norm)
        return dx.reshape(shape), None, None, None, None


def swdft2d_backward(dy: torch.Tensor, N0: int, N1: int, dtype=torch.float32, norm: str = "none",
                     algo: str = "auto") -> torch.Tensor:
    """Adjoint: dy [B,P0,P1,n0,n1] -> dx [B,N0,N1] (Re of M^H dy for real dtypes)."""
    squeeze = dy.dim() == 4
    dyb = dy.unsqueeze(0) if squeeze else dy
    B, P0, P1, n0, n1 = dyb.shape
    dx = _cached_plan(N0, N1, n0, n1, dtype, B, norm, algo).backward(dyb.contiguous())
    return dx[0] if squeeze else dx


class SWDFT2dFn(torch.autograd.Function):
    """y = swdft2d(x); the backward pass runs the library's adjoint kernel.

    For real x and a real loss L, PyTorch hands backward the conjugate
    Wirtinger gradient dL/dRe(y) + i dL/dIm(y); the gradient with respect to x
    is Re(M^H of it), which is what the adjoint computes.
    """

    @staticmethod
    def forward(ctx, x, n0, n1, norm="none"):
        ctx.meta = (x.shape, x.dtype, n0, n1, norm)
        return swdft2d(x, n0, n1, norm=norm)

    @staticmethod
    def backward(ctx, gy):
        shape, dtype, n0, n1, norm = ctx.meta
        N0, N1 = shape[-2], shape[-1]
        dx = swdft2d_backward(gy.contiguous(), N0, N1, dtype=dtype, norm=norm)
        return dx.reshape(shape), None, None, None


def read_probe(buf: torch.Tensor, sink: torch.Tensor | None = None) -> None:
    """Read buf with non-temporal 16-byte loads (HBM read-ceiling probe); sink
    is a device float32 tensor that is written only if the values read sum to
    one particular NaN."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("probe buffer must be a contiguous cuda tensor")
    if sink is None:
        sink = torch.empty(1, dtype=torch.float32, device=buf.device)
    with torch.cuda.device(buf.device):
        stream = torch.cuda.current_stream(buf.device).cuda_stream
        check(lib.swdft2d_read_probe(buf.data_ptr(), buf.numel() * buf.element_size(),
                                     sink.data_ptr(), stream), "swdft2d_read_probe")


def write_probe(buf: torch.Tensor, nbytes: int | None = None) -> None:
    """Fill buf with a constant using a memset-like pattern (HBM write-ceiling probe)."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("probe buffer must be a contiguous cuda tensor")
    nbytes = buf.numel() * buf.element_size() if nbytes is None else nbytes
    with torch.cuda.device(buf.device):
        stream = torch.cuda.current_stream(buf.device).cuda_stream
        check(lib.swdft2d_write_probe(buf.data_ptr(), nbytes, stream), "swdft2d_write_probe")
