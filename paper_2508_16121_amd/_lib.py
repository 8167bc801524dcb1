"""ctypes loader for libsvdlut.so.

torch is imported first so that its HIP runtime (same SONAME as the one the library links)
is the one already resident in the process; the library then binds to it and shares its
streams and allocations.  A missing library raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsvdlut.so")

F32, F16 = 0, 1
LOSS_L1, LOSS_MSE = 0, 1
STATUS = {0: "SVDLUT_OK", 1: "SVDLUT_EINVAL", 2: "SVDLUT_EUNSUPPORTED", 3: "SVDLUT_ENOMEM", 4: "SVDLUT_EDEVICE"}

# public symbols of include/svdlut.h with their ctypes signatures
P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
SZ = C.c_size_t
FL = C.c_float
SIGS = {
    "svdlut_last_error": (C.c_char_p, []),
    "svdlut_version": (C.c_char_p, []),
    "svdlut_reconstruct": (I32, [P, P, P, P, I32, I32, I32, P]),
    "svdlut_apply": (I32, [P, P, I32, P, P, P, P, I32, P, I32, I32, I32, I32, I32, I32, I32, P]),
    "svdlut_apply_grid": (I32, [P, P, I32, P, P, P, P, I32, P, P, P, P, I32, I32,
                                I32, I32, I32, I32, I32, I32, I32, P]),
    "svdlut_apply_bwd_workspace_size": (SZ, [I32, I32]),
    "svdlut_apply_grid_bwd_workspace_size": (SZ, [I32, I32, I32]),
    "svdlut_unfused_workspace_size": (SZ, [I32, I32, I32, I32, I32]),
    "svdlut_unfused_apply": (I32, [P, P, P, P, P, P, P, P, I32, I32, I32, I32, I32, I32, P, SZ, P]),
    "svdlut_apply_grid_bwd": (I32, [P, P, I32, P, P, P, P, I32, P, P, I32, I32, P, P, P, P, P, P, P, P, P,
                                    I32, I32, I32, I32, I32, I32, I32, P, SZ, P]),
    "svdlut_apply_bwd": (I32, [P, P, I32, P, P, P, P, I32, P, P, P, P, P, P,
                               I32, I32, I32, I32, I32, I32, I32, P, SZ, P]),
    "svdlut_apply_bwd_noalloc": (I32, [P, P, I32, P, P, P, P, I32, P, P, P, P, P, P,
                                       I32, I32, I32, I32, I32, I32, I32, P]),
    "svdlut_set_deterministic": (None, [I32]),
    "svdlut_get_deterministic": (I32, []),
    "svdlut_deterministic_workspace_size": (SZ, [I32, I32, I32, I32, I32]),
    "svdlut_plan_create": (I32, [P, I32, I32, I32, I32, I32, P]),
    "svdlut_plan_autotune": (I32, [P, P, P, P, P, P, P, P, P]),
    "svdlut_plan_launch": (I32, [P, P, P, P, P, P, P, P, P]),
    "svdlut_plan_launch_direct": (I32, [P, P, P, P, P, P, P, P, P]),
    "svdlut_plan_set_shape": (I32, [P, I32, I32, I32]),
    "svdlut_plan_get_info": (I32, [P, P]),
    "svdlut_plan_destroy": (I32, [P]),
    "svdlut_loss_workspace_size": (SZ, [I64]),
    "svdlut_loss": (I32, [P, P, I32, I64, I32, P, P, P, SZ, P]),
    "svdlut_generator_param_count": (SZ, [I32, I32]),
    "svdlut_generator_workspace_size": (SZ, [I32, I32, I32]),
    "svdlut_generator_fwd": (I32, [P, P, I32, I32, I32, I32, I32, I32, P, P, P, P, P, SZ, P]),
    "svdlut_generator_bwd": (I32, [P, P, P, P, P, P, I32, I32, I32, P, SZ, P]),
    "svdlut_apply_loss_bwd_workspace_size": (SZ, [I32, I32]),
    "svdlut_apply_loss_bwd": (I32, [P, P, I32, P, P, P, P, I32, P, I32, P, P, P, P, P, P, P, I32, I32, I32, I32, I32,
                                    I32, I32, P, SZ, P]),
    "svdlut_lut3d_workspace_size": (SZ, [I32, I32]),
    "svdlut_lut3d_apply": (I32, [P, P, P, I32, I32, I32, I32, P, SZ, P]),
    "svdlut_lut1d_apply": (I32, [P, P, P, I32, I32, I32, I32, P]),
    "svdlut_paper_generator_param_count": (SZ, [I32, I32, I32, I32]),
    "svdlut_paper_generator_workspace_size": (SZ, [I32, I32, I32, I32, I32]),
    "svdlut_paper_generator_fwd": (I32, [P, P, I32, I32, I32, I32, I32, I32, I32, I32, P, P, P, P, P, P, P, P, P,
                                         P, SZ, P]),
    "svdlut_paper_generator_bwd": (I32, [P, P, P, P, P, P, P, P, P, P, P, I32, I32, I32, I32, I32, P, SZ, P]),
    "svdlut_adam_step": (I32, [P, P, P, P, I64, FL, FL, FL, FL, I32, P]),
}


class ImageDesc(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("h", C.c_int32), ("w", C.c_int32),
                ("x_off", C.c_int64), ("y_off", C.c_int64), ("map_off", C.c_int64)]


class PlanInfo(C.Structure):
    _fields_ = [("pixels", C.c_int64), ("tiles", C.c_int64), ("block", C.c_int32),
                ("grid", C.c_int32), ("tuned", C.c_int32), ("graph", C.c_int32),
                ("tile_px", C.c_int32), ("px_per_lane", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("reserved", C.c_int32)]


class SvdlutError(RuntimeError):
    pass


_lib = None


def load(path: str = LIB_PATH):
    """Load libsvdlut.so (once) and attach the signatures of every public symbol."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_2508_16121_amd/build.py`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGS.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, what: str):
    if status != 0:
        msg = load().svdlut_last_error().decode(errors="replace")
        raise SvdlutError(f"{what}: {STATUS.get(status, status)}: {msg}")
