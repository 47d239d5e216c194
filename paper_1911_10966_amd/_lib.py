"""ctypes declarations of the C ABI in include/sbp.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsbp_hip.so")

SBP_OK = 0
SBP_ERR_ARG = -1
SBP_ERR_DEGREE = -2
SBP_ERR_MESH = -3
SBP_ERR_NONPHYSICAL = -4
SBP_ERR_HIP = -5
SBP_ERR_WORKSPACE = -6
SBP_ERR_SCRATCH = -7
SBP_NOALLOC_SCRATCH_BYTES = 64 << 20
SBP_NOALLOC_MAX_PROBLEMS = 16
SBP_PROFILE_SLOTS = 4096
SBP_MAX_P = 15
SBP_MAX_VJP_P = 8
SBP_BC_DIRICHLET = -1
SBP_BC_SLIP_WALL = -2
SBP_BC_ADIABATIC_WALL = -3

EXPORTED = ("sbp_version", "sbp_error_string", "sbp_lgl_operator", "sbp_metrics",
            "sbp_workspace_bytes", "sbp_residual", "sbp_rk_step", "sbp_residual_vjp",
            "sbp_profile_residual", "sbp_autotune", "sbp_schedule_count", "sbp_set_schedule",
            "sbp_status", "sbp_release", "sbp_residual_noalloc", "sbp_profile_collect",
            "sbp_metrics_optimized")


class sbp_problem(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_int32),
        ("iface_diss", ctypes.c_int32),
        ("n_elem", ctypes.c_int64),
        ("nbr", ctypes.c_void_p),
        ("metric", ctypes.c_void_p),
        ("jac", ctypes.c_void_p),
        ("gamma", ctypes.c_double),
        ("R", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("Pr", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("two_point", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("bc_state", ctypes.c_void_p),
        ("source", ctypes.c_void_p),
        ("face_orient", ctypes.c_void_p),
    ]


class SBPError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {error_string(code)} (code {code})")


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run python -m paper_1911_10966_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        P = ctypes.POINTER(sbp_problem)
        dp = ctypes.POINTER(ctypes.c_double)
        L.sbp_version.restype = ctypes.c_int
        L.sbp_error_string.argtypes = [ctypes.c_int]
        L.sbp_error_string.restype = ctypes.c_char_p
        L.sbp_lgl_operator.argtypes = [i32, dp, dp, dp]
        L.sbp_metrics.argtypes = [i32, i64, vp, vp, vp, vp]
        L.sbp_metrics_optimized.argtypes = [i32, i64, vp, vp, vp, vp, vp]
        L.sbp_workspace_bytes.argtypes = [P, i32]
        L.sbp_workspace_bytes.restype = sz
        L.sbp_residual.argtypes = [P, i32, vp, vp, vp, sz, vp]
        L.sbp_rk_step.argtypes = [P, i32, vp, vp, i32, vp, sz, vp]
        L.sbp_residual_vjp.argtypes = [P, i32, vp, vp, vp, vp, sz, vp]
        L.sbp_status.argtypes = [vp, vp, ctypes.POINTER(i32)]
        L.sbp_release.argtypes = [vp]
        L.sbp_residual_noalloc.argtypes = [P, i32, vp, vp, vp, vp]
        L.sbp_schedule_count.argtypes = [i32]
        L.sbp_set_schedule.argtypes = [P, i32, vp, sz, i32, i32]
        L.sbp_autotune.argtypes = [P, i32, vp, vp, vp, sz, vp, i32, ctypes.POINTER(i32)]
        L.sbp_profile_residual.argtypes = [P, i32, vp, vp, vp, sz, vp, ctypes.POINTER(ctypes.c_float)]
        L.sbp_profile_collect.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


def error_string(code: int) -> str:
    try:
        return lib().sbp_error_string(code).decode()
    except Exception:  # pragma: no cover - library missing
        return f"error {code}"


def check(code: int, where: str):
    if code != SBP_OK:
        raise SBPError(code, where)
