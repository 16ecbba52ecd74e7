"""ctypes view of librsv.so (the C ABI declared in include/rsv.h).

Argument marshalling only.  Loading fails loudly when the library has not been
built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librsv.so")

RSV_U8, RSV_F32 = 0, 1
RSV_MAX_D = 512
RSV_ADJOINT_NOALLOC_MAX_PIXELS = 1 << 21
RSV_PLANE_MAX_K = 1024

STATUS = {0: "RSV_OK", -1: "RSV_E_NULL", -2: "RSV_E_SHAPE", -3: "RSV_E_PARAM",
          -4: "RSV_E_DTYPE", -5: "RSV_E_ALIGN", -6: "RSV_E_HIP", -7: "RSV_E_NOMEM"}


class RsvError(RuntimeError):
    def __init__(self, status: int, where: str, message: str = ""):
        self.status = status
        name = STATUS.get(status, str(status))
        super().__init__(f"{where}: {name} ({message})")


class Image(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("height", C.c_int32),
                ("width", C.c_int32), ("pitch", C.c_int64)]


class Plane(C.Structure):
    _fields_ = [("a0", C.c_double), ("a1", C.c_double), ("a2", C.c_double), ("delta", C.c_double)]


class Camera(C.Structure):
    _fields_ = [("f", C.c_double), ("baseline", C.c_double), ("u0", C.c_double), ("v0", C.c_double)]


class Params(C.Structure):
    _fields_ = [("D", C.c_int32), ("block_radius", C.c_int32), ("agg_radius", C.c_int32),
                ("lr_threshold", C.c_int32), ("gamma_d", C.c_float), ("gamma_r", C.c_float),
                ("sigma_min", C.c_float)]


_P = C.c_void_p
_SIGNATURES = {
    "rsv_warp": (C.c_int, [Image, Plane, _P, _P]),
    "rsv_cost_volume": (C.c_int, [Image, _P, C.POINTER(Params), _P, _P, _P]),
    "rsv_cost_volume_joint": (C.c_int, [Image, _P, C.POINTER(Params), _P, C.c_int64, _P]),
    "rsv_aggregate": (C.c_int, [_P, Image, C.POINTER(Params), _P, _P]),
    "rsv_aggregate_strided": (C.c_int, [_P, C.c_int64, C.c_int64, Image, C.POINTER(Params), _P, _P]),
    "rsv_aggregate_argmax": (C.c_int, [_P, C.c_int64, C.c_int64, Image, C.POINTER(Params), _P, _P]),
    "rsv_aggregate_select": (C.c_int, [_P, C.c_int64, C.c_int64, Image, C.POINTER(Params), _P, _P, _P, _P,
                                       _P]),
    "rsv_aggregate_views": (C.c_int, [_P, C.c_int64, C.c_int64, _P, C.c_int64, C.c_int64, Image, Image,
                                      C.POINTER(Params), _P, _P, _P, _P]),
    "rsv_lr_check": (C.c_int, [_P, _P, C.c_int32, C.c_int32, C.c_int32, _P, _P]),
    "rsv_cost_argmax_views": (C.c_int, [_P, C.c_int64, C.c_int64, _P, C.c_int64, C.c_int64, C.c_int32, C.c_int32,
                                        C.c_int32, _P, _P, _P]),
    "rsv_aggregate_restricted_views": (C.c_int, [_P, C.c_int64, C.c_int64, _P, C.c_int64, C.c_int64, Image, Image,
                                                 C.POINTER(Params), _P, _P, C.c_int32, _P, _P, _P, _P]),
    "rsv_select_subpixel": (C.c_int, [_P, _P, C.c_int32, C.c_int32, C.POINTER(Params), _P, _P, _P,
                                      _P, _P, _P]),
    "rsv_select_subpixel_ref": (C.c_int, [_P, _P, C.c_int32, C.c_int32, C.POINTER(Params), _P, _P, _P, _P,
                                          _P]),
    "rsv_cost_argmax": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_int32, _P, _P]),
    "rsv_aggregate_restricted_argmax": (C.c_int, [_P, C.c_int64, C.c_int64, Image, C.POINTER(Params), _P,
                                                  C.c_int32, _P, _P]),
    "rsv_aggregate_restricted_select": (C.c_int, [_P, C.c_int64, C.c_int64, Image, C.POINTER(Params), _P,
                                                  C.c_int32, _P, _P, _P, _P, _P]),
    "rsv_plane_ransac_workspace_bytes": (C.c_size_t, [C.c_int32]),
    "rsv_plane_ransac": (C.c_int, [_P, _P, C.c_int32, C.c_int32, _P, C.c_int32, C.c_float, _P, _P, _P, _P,
                                   _P]),
    "rsv_triangulate": (C.c_int, [_P, _P, C.c_int32, C.c_int32, Plane, Camera, _P, _P, _P]),
    "rsv_selected_cost_sum": (C.c_int, [_P, _P, _P, C.c_int32, C.c_int32, C.c_int32, _P, _P]),
    "rsv_cost_adjoint_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "rsv_selected_aggregate_sum": (C.c_int, [_P, C.c_int64, C.c_int64, Image, C.POINTER(Params), _P, _P,
                                             _P, _P]),
    "rsv_cost_adjoint": (C.c_int, [Image, Image, Plane, C.POINTER(Params), _P, C.c_int64, C.c_int64, _P,
                                   _P, _P, _P, _P, _P, _P, _P]),
    "rsv_cost_adjoint_noalloc": (C.c_int, [Image, Image, Plane, C.POINTER(Params), _P, C.c_int64, C.c_int64,
                                           _P, _P, _P, _P, _P, _P, _P]),
    "rsv_tuning_default": (None, [_P]),
    "rsv_batch_plan_create": (C.c_int, [_P, C.c_int32, C.POINTER(Params), _P, _P]),
    "rsv_batch_run": (C.c_int, [_P, _P]),
    "rsv_batch_plan_info": (C.c_int, [_P, _P, _P, _P]),
    "rsv_batch_plan_destroy": (C.c_int, [_P]),
    "rsv_autotune": (C.c_int, [_P, C.c_int32, C.POINTER(Params), _P, _P, _P]),
    "rsv_status_string": (C.c_char_p, [C.c_int]),
    "rsv_last_hip_error": (C.c_int, []),
    "rsv_version": (C.c_int, []),
}

_lib = None


def load(path: str | None = None):
    """Load librsv.so once; raises OSError if it is missing or lacks a symbol."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise OSError(f"librsv.so not built ({p}); run `python -m paper_1807_07433_amd.build`")
    lib = C.CDLL(p)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)  # AttributeError if the symbol is missing
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_symbols() -> list[str]:
    return list(_SIGNATURES)


def check(status: int, where: str):
    if status != 0:
        lib = load()
        msg = lib.rsv_status_string(status).decode()
        if status == -6:
            msg += f"; hipError {lib.rsv_last_hip_error()}"
        raise RsvError(status, where, msg)
