"""ctypes declarations of the C ABI in include/stencil.h (argument marshalling
only; every step of the computation runs in libstencil's HIP kernels).

The library must have been built (``python -m paper_2609_06694_amd.build`` or
``__graft_entry__.build()``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# STENCIL_LIBRARY may name another build of the same library (same ABI).
LIB_PATH = os.environ.get("STENCIL_LIBRARY") or os.path.join(HERE, "libstencil.so")

ST_OK, ST_EINVAL, ST_ESHAPE, ST_EUNSUPPORTED, ST_EWORKSPACE, ST_EHIP, ST_ENOMEM, ST_ETUNE = range(8)
STATUS_NAMES = {0: "ST_OK", 1: "ST_EINVAL", 2: "ST_ESHAPE", 3: "ST_EUNSUPPORTED", 4: "ST_EWORKSPACE",
                5: "ST_EHIP", 6: "ST_ENOMEM", 7: "ST_ETUNE"}
ST_F32, ST_F16, ST_F64 = 0, 1, 2
ST_PERIODIC, ST_ZERO = 0, 1
ST_STAR, ST_BOX = 0, 1
ST_LINEAR, ST_WAVE, ST_VARCOEF = 0, 1, 2
ST_VARIANT_AUTO, ST_VARIANT_TB2D, ST_VARIANT_ZM3D, ST_VARIANT_WAVE3D, ST_VARIANT_WAVE3D_LDS = 0, 1, 2, 3, 4
ST_VARIANT_YM2D = 5
ST_VARIANT_ZM3D_MFMA = 6
ST_VARIANT_ZM3D_H2 = 8
ST_VARIANT_YM2D_H2 = 9
ST_VARIANT_YM3D = 10
VARIANT_NAMES = {0: "auto", 1: "tb2d", 2: "zm3d", 3: "wave3d", 4: "wave3d_lds", 5: "ym2d", 6: "zm3d_mfma",
                 7: "vc3d", 8: "zm3d_h2", 9: "ym2d_h2", 10: "ym3d"}

# Every symbol the header declares; tests check the library exports them all.
EXPORTED = ["stencil_plan", "stencil_plan_destroy", "stencil_workspace_bytes",
            "stencil_plan_describe", "stencil_plan_describe_reverse", "stencil_plan_describe_batched",
            "stencil_plan_coefficients", "stencil_apply", "stencil_apply_adjoint",
            "stencil_apply_varcoef", "stencil_apply_varcoef_adjoint",
            "stencil_wave_gradient", "stencil_plan_batched", "stencil_apply_batched",
            "stencil_autotune", "stencil_autotune_stats", "stencil_last_error", "stencil_version",
            "stencil_apply_noalloc", "stencil_noalloc_capacity"]


class StProblem(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int64 * 3), ("shape", ctypes.c_int32),
                ("radius", ctypes.c_int32), ("coeffs", ctypes.POINTER(ctypes.c_float)),
                ("dtype", ctypes.c_int32), ("boundary", ctypes.c_int32), ("update", ctypes.c_int32)]


class StPlanOpts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("tsteps", ctypes.c_int32), ("zchunk", ctypes.c_int32), ("ckpt_every", ctypes.c_int32)]


class StWaveArgs(ctypes.Structure):
    _fields_ = [("u_prev", ctypes.c_void_p), ("kappa", ctypes.c_void_p), ("src", ctypes.c_int64 * 3),
                ("wavelet", ctypes.c_void_p), ("rec_z", ctypes.c_int64), ("traces", ctypes.c_void_p),
                ("target", ctypes.c_void_p), ("sponge_width", ctypes.c_int32), ("sponge_strength", ctypes.c_float)]


class StencilError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """Load libstencil.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the HIP library is the only compute path)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, sz = ctypes.c_int32, ctypes.c_size_t
    L.stencil_plan.argtypes = [ctypes.POINTER(StProblem), ctypes.POINTER(StPlanOpts), ctypes.POINTER(P)]
    L.stencil_plan.restype = ctypes.c_int
    L.stencil_plan_destroy.argtypes = [P]
    L.stencil_plan_destroy.restype = None
    L.stencil_workspace_bytes.argtypes = [P, i32, i32]
    L.stencil_workspace_bytes.restype = sz
    ip = ctypes.POINTER(i32)
    L.stencil_plan_describe.argtypes = [P, ip, ip, ip, ip, ip]
    L.stencil_plan_describe.restype = ctypes.c_int
    L.stencil_plan_describe_reverse.argtypes = [P, ip, ip, ip, ip, ip]
    L.stencil_plan_describe_reverse.restype = ctypes.c_int
    L.stencil_plan_describe_batched.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ip, ip,
                                                ctypes.POINTER(ctypes.c_int64)]
    L.stencil_plan_describe_batched.restype = ctypes.c_int
    L.stencil_plan_coefficients.argtypes = [P, ctypes.POINTER(ctypes.c_float), i32,
                                            ctypes.POINTER(ctypes.c_double)]
    L.stencil_plan_coefficients.restype = ctypes.c_int
    L.stencil_apply.argtypes = [P, P, P, i32, ctypes.POINTER(StWaveArgs), P, sz, P]
    L.stencil_apply.restype = ctypes.c_int
    L.stencil_apply_noalloc.argtypes = [P, P, P, i32, ctypes.POINTER(StWaveArgs), P]
    L.stencil_apply_noalloc.restype = ctypes.c_int
    L.stencil_noalloc_capacity.argtypes = []
    L.stencil_noalloc_capacity.restype = sz
    L.stencil_apply_adjoint.argtypes = [P, P, P, i32, ctypes.POINTER(StWaveArgs), P, sz, P]
    L.stencil_apply_adjoint.restype = ctypes.c_int
    L.stencil_apply_varcoef.argtypes = [P, P, P, P, i32, P, sz, P]
    L.stencil_apply_varcoef.restype = ctypes.c_int
    L.stencil_apply_varcoef_adjoint.argtypes = [P, P, P, P, i32, P, sz, P]
    L.stencil_apply_varcoef_adjoint.restype = ctypes.c_int
    L.stencil_wave_gradient.argtypes = [P, P, ctypes.POINTER(StWaveArgs), i32, P, P, P, sz, P]
    L.stencil_wave_gradient.restype = ctypes.c_int
    L.stencil_plan_batched.argtypes = [ctypes.POINTER(StProblem), i32, ctypes.POINTER(StPlanOpts),
                                       ctypes.POINTER(P)]
    L.stencil_plan_batched.restype = ctypes.c_int
    L.stencil_apply_batched.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), i32, P, sz, P]
    L.stencil_apply_batched.restype = ctypes.c_int
    L.stencil_autotune.argtypes = [P, P, sz, P]
    L.stencil_autotune.restype = ctypes.c_int
    L.stencil_autotune_stats.argtypes = [P, ip, ip]
    L.stencil_autotune_stats.restype = ctypes.c_int
    L.stencil_last_error.argtypes = []
    L.stencil_last_error.restype = ctypes.c_char_p
    L.stencil_version.argtypes = []
    L.stencil_version.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status: int) -> None:
    if status != ST_OK:
        raise StencilError(status, lib().stencil_last_error().decode())
