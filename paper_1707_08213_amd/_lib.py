"""ctypes binding of libswdft2d.so (the C ABI declared in include/swdft2d.h).

Argument marshalling only: every step of the transform runs in the library's
HIP kernels. If the library has not been built this module raises on import;
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIBRARY = os.path.join(PKG, "libswdft2d.so")

SWDFT_R32, SWDFT_C32, SWDFT_R64, SWDFT_C64 = 0, 1, 2, 3
SWDFT_NORM_NONE, SWDFT_NORM_ORTHO = 0, 1
(SWDFT_ALGO_AUTO, SWDFT_ALGO_TREE, SWDFT_ALGO_DENSE_BF16X2, SWDFT_ALGO_DIRECT_F64,
 SWDFT_ALGO_SWFFT) = 0, 1, 2, 3, 4

STATUS = {
    0: "SWDFT_OK", 1: "SWDFT_E_ARG", 2: "SWDFT_E_NOT_POW2", 3: "SWDFT_E_WINDOW",
    4: "SWDFT_E_DTYPE", 5: "SWDFT_E_OVERFLOW", 6: "SWDFT_E_NOMEM", 7: "SWDFT_E_ALIGN",
    8: "SWDFT_E_DEVICE", 9: "SWDFT_E_PLAN",
}
STATUS_CODE = {v: k for k, v in STATUS.items()}

class Desc(ctypes.Structure):
    """swdft2d_desc_t"""
    _fields_ = [("N0", ctypes.c_int64), ("N1", ctypes.c_int64), ("n0", ctypes.c_int32),
                ("n1", ctypes.c_int32), ("x_offset", ctypes.c_int64), ("y_offset", ctypes.c_int64)]


# name -> (restype, argtypes), the full exported surface
_i64, _i32, _vp, _int = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int
_PLAN_P = ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = {
    "swdft2d_plan": (_int, [_PLAN_P, _i64, _i64, _i32, _i32, _int, _i64]),
    "swdft2d_set_norm": (_int, [_vp, _int]),
    "swdft2d_set_algo": (_int, [_vp, _int]),
    "swdft2d_exec": (_int, [_vp, _vp, _vp, _vp]),
    "swdft2d_backward": (_int, [_vp, _vp, _vp, _vp]),
    "swdft2d_backward_noalloc": (_int, [_vp, _vp, _vp, _vp]),
    "swdft2d_destroy": (_int, [_vp]),
    "swdft2d_output_elems": (_i64, [_vp]),
    "swdft2d_output_bytes": (_i64, [_vp]),
    "swdft2d_describe": (_int, [_vp, ctypes.c_char_p, _i32]),
    "swdft2d_status_string": (ctypes.c_char_p, [_int]),
    "swdft2d_last_error": (ctypes.c_char_p, []),
    "swdft2d_write_probe": (_int, [_vp, _i64, _vp]),
    "swdft2d_read_probe": (_int, [_vp, _i64, _vp, _vp]),
    "swdft2d_twiddles": (_int, [_vp, _i32, ctypes.POINTER(ctypes.c_float), _i32]),
    "swdft2d_plan_batched": (_int, [_PLAN_P, _vp, _i64, _int]),
    "swdft2d_tune": (_int, [_vp, _vp, _vp, _vp]),
    "swdft2d_stream_create": (_int, [_PLAN_P, _i64, _i32, _i32, _int]),
    "swdft2d_stream_set_norm": (_int, [_vp, _int]),
    "swdft2d_stream_rows": (_i64, [_vp]),
    "swdft2d_stream_completes": (_i64, [_vp, _i64]),
    "swdft2d_stream_push": (_int, [_vp, _vp, _i64, _vp, _vp]),
    "swdft2d_stream_reset": (_int, [_vp, _vp]),
    "swdft2d_stream_destroy": (_int, [_vp]),
    "swdft3d_plan": (_int, [_PLAN_P, _i64, _i64, _i64, _i32, _i32, _i32, _int, _i64]),
    "swdft3d_set_norm": (_int, [_vp, _int]),
    "swdft3d_backward": (_int, [_vp, _vp, _vp, _vp]),
    "swdft3d_exec": (_int, [_vp, _vp, _vp, _vp]),
    "swdft3d_output_elems": (_i64, [_vp]),
    "swdft3d_describe": (_int, [_vp, ctypes.c_char_p, _i32]),
    "swdft3d_destroy": (_int, [_vp]),
}


class SwdftError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        self.name = STATUS.get(status, f"status {status}")
        super().__init__(f"{where}: {self.name}: {detail}")


def _load():
    if not os.path.exists(LIBRARY):
        raise ImportError(
            f"{LIBRARY} is missing: build it with `python paper_1707_08213_amd/build.py` "
            "(the HIP library is required; there is no CPU fallback)")
    lib = ctypes.CDLL(LIBRARY)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(status: int, where: str) -> None:
    if status != 0:
        detail = lib.swdft2d_last_error()
        raise SwdftError(status, where, detail.decode() if detail else "")
