"""ctypes declarations of the C-ABI in include/wlseno.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwlseno.so")

WLSENO_OK = 0
WLSENO_ENUMERIC = 6
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "EUNSUPPORTED", 6: "ENUMERIC"}
FLUX = {"advection": 0, "burgers": 1, "euler": 2}
MESH_PERIODIC_1D = 1
MESH_PERIODIC_2D = 2

# every symbol include/wlseno.h declares
EXPORTS = [
    "wlseno_params_default", "wlseno_create", "wlseno_destroy", "wlseno_last_error", "wlseno_set_stream",
    "wlseno_mesh_upload", "wlseno_stencil_build", "wlseno_get_info", "wlseno_get_stencil",
    "wlseno_reconstruct", "wlseno_rhs", "wlseno_step", "wlseno_last_alpha", "wlseno_time_kernel",
    "wlseno_batch_add_mesh", "wlseno_batch_step", "wlseno_batch_last_alpha", "wlseno_set_graphs",
    "wlseno_rhs_vjp", "wlseno_step_adjoint", "wlseno_step_record", "wlseno_step_adjoint_recorded",
    "wlseno_rhs_noalloc", "wlseno_set_step_mode", "wlseno_autotune", "wlseno_batch_params",
    "wlseno_set_numeric_check",
]


class Params(C.Structure):
    _fields_ = [
        ("p", C.c_int32), ("n_lo", C.c_int32), ("n_hi", C.c_int32), ("flux", C.c_int32),
        ("weight_mode", C.c_int32), ("lanes", C.c_int32),
        ("eps", C.c_double), ("alpha_w", C.c_double), ("rank_tol", C.c_double),
        ("velocity", C.c_double * 3), ("gamma", C.c_double), ("bc", C.c_int32), ("characteristic", C.c_int32), ("far_state", C.c_double * 5), ("balance", C.c_int32), ("lf_alpha", C.c_int32), ("h_mode", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("m", C.c_int32), ("n_vars", C.c_int32), ("faces_per_cell", C.c_int32),
        ("points_per_face", C.c_int32), ("min_stencil", C.c_int32), ("max_stencil", C.c_int32),
        ("n_mesh", C.c_int32), ("n_cell", C.c_int64), ("nnz", C.c_int64), ("h", C.c_double),
        ("min_insphere", C.c_double),
    ]


class Tune(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("lanes", C.c_int32 * 4), ("us", C.c_double * 4), ("chosen", C.c_int32),
        ("cached", C.c_int32),
    ]


class LibraryMissing(RuntimeError):
    pass


_lib = None


def load():
    """Load libwlseno.so (built in-tree); raise if it is not there."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(
            f"{LIB_PATH} is missing: build it with `python -m paper_1602_02694_amd.build` "
            "(there is no fallback implementation)")
    lib = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    lib.wlseno_params_default.argtypes = [C.POINTER(Params)]
    lib.wlseno_params_default.restype = None
    lib.wlseno_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
    lib.wlseno_set_numeric_check.argtypes = [vp, C.c_int]
    lib.wlseno_destroy.argtypes = [vp]
    lib.wlseno_last_error.argtypes = [vp]
    lib.wlseno_last_error.restype = C.c_char_p
    lib.wlseno_set_stream.argtypes = [vp, vp]
    lib.wlseno_mesh_upload.argtypes = [vp, C.c_int, C.c_int64, dp, C.c_int64, ip, C.c_uint32]
    lib.wlseno_stencil_build.argtypes = [vp, C.POINTER(Params)]
    lib.wlseno_get_info.argtypes = [vp, C.POINTER(Info)]
    lib.wlseno_get_stencil.argtypes = [vp, ip, ip]
    lib.wlseno_reconstruct.argtypes = [vp, vp, vp, vp, vp]
    lib.wlseno_rhs.argtypes = [vp, vp, vp]
    lib.wlseno_rhs_noalloc.argtypes = [vp, vp, vp]
    lib.wlseno_step.argtypes = [vp, vp, C.c_double, C.c_int]
    lib.wlseno_last_alpha.argtypes = [vp, dp]
    lib.wlseno_time_kernel.argtypes = [vp, C.c_int, vp, C.c_int, dp]
    lib.wlseno_batch_add_mesh.argtypes = [vp, C.c_int, C.c_int64, dp, C.c_int64, ip, C.POINTER(C.c_int32)]
    lib.wlseno_batch_step.argtypes = [vp, vp, dp, C.c_int]
    lib.wlseno_batch_last_alpha.argtypes = [vp, dp]
    lib.wlseno_set_graphs.argtypes = [vp, C.c_int]
    lib.wlseno_set_step_mode.argtypes = [vp, C.c_int]
    lib.wlseno_autotune.argtypes = [vp, vp, C.POINTER(Tune)]
    lib.wlseno_batch_params.argtypes = [vp, C.c_int, C.POINTER(Params)]
    lib.wlseno_rhs_vjp.argtypes = [vp, vp, vp, vp]
    lib.wlseno_step_adjoint.argtypes = [vp, vp, C.c_double, C.c_int, C.c_int, vp, vp]
    lib.wlseno_step_record.argtypes = [vp, vp, C.c_double, C.c_int, C.c_int]
    lib.wlseno_step_adjoint_recorded.argtypes = [vp, vp, vp]
    for name in EXPORTS:
        f = getattr(lib, name)
        if name not in ("wlseno_params_default", "wlseno_last_error"):
            f.restype = C.c_int
    _lib = lib
    return lib
