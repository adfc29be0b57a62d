"""ctypes binding of libswe_hweno.so (the C ABI declared in include/swe_hweno.h).

Argument marshalling only: every step of the solver runs in the library's HIP kernels. The
library is loaded from this package directory; if it is missing the import fails loudly (there
is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswe_hweno.so")

OK, EINVAL, ENOMEM, EHIP, EDRY, ENONFINITE = 0, -1, -2, -3, -4, -5
BC_PERIODIC, BC_REFLECTIVE = 0, 1
FIXED_DT, FIXED_ALPHA, NO_LIMITER, CHECK_DRY = 1, 2, 4, 8
ABI_VERSION = 1

# every symbol include/swe_hweno.h declares
EXPORTS = ("swe_hweno_init", "swe_hweno_rhs", "swe_hweno_limit", "swe_hweno_alpha", "swe_hweno_step",
           "swe_hweno_run", "swe_hweno_sync", "swe_hweno_destroy", "swe_hweno_strerror", "swe_hweno_abi_version",
           "swe_hweno_tile", "swe_hweno_set_timing", "swe_hweno_get_timing", "swe_hweno_ctx_tile",
           "swe_hweno_batch_init", "swe_hweno_batch_run", "swe_hweno_batch_set_rows", "swe_hweno_batch_autotune",
           "swe_hweno_batch_sync", "swe_hweno_batch_destroy", "swe_hweno_batch_tune_cache_size",
           "swe_hweno_batch_tune_cache_clear",
           "swe_hweno_init_f32", "swe_hweno_rhs_f32", "swe_hweno_limit_f32", "swe_hweno_alpha_f32",
           "swe_hweno_step_f32", "swe_hweno_run_f32",
           "swe_hweno_rhs_vjp", "swe_hweno_limit_vjp", "swe_hweno_run_vjp", "swe_hweno_bottom_slopes",
           "swe_hweno_bottom_slopes_vjp", "swe_hweno_run_checkpointed", "swe_hweno_run_vjp_checkpointed",
           "swe_hweno_step_noalloc", "swe_hweno_noalloc_capacity", "swe_hweno_math_check",
           "swe_hweno_source_hash")


class SweError(RuntimeError):
    def __init__(self, code, where=""):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})" if where else f"{strerror(code)} ({code})")


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("g", ctypes.c_double), ("cfl", ctypes.c_double), ("eps", ctypes.c_double),
        ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int), ("flags", ctypes.c_int),
        ("fixed_dt", ctypes.c_double), ("alpha_x", ctypes.c_double), ("alpha_y", ctypes.c_double),
    ]


class Instance(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
        ("b", ctypes.c_void_p), ("bx", ctypes.c_void_p), ("by", ctypes.c_void_p), ("state", ctypes.c_void_p),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc for gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, I, D = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER(Params)
    sig = {
        "swe_hweno_init": (I, [P, dp, dp, dp, vp, ctypes.POINTER(vp)]),
        "swe_hweno_rhs": (I, [vp, dp, dp, D, D]),
        "swe_hweno_limit": (I, [vp, dp, dp]),
        "swe_hweno_alpha": (I, [vp, dp, ctypes.POINTER(D)]),
        "swe_hweno_step": (I, [vp, dp, D, ctypes.POINTER(D)]),
        "swe_hweno_run": (I, [vp, dp, I, D, ctypes.POINTER(D), ctypes.POINTER(I)]),
        "swe_hweno_init_f32": (I, [P, dp, dp, dp, vp, ctypes.POINTER(vp)]),
        "swe_hweno_rhs_f32": (I, [vp, dp, dp, D, D]),
        "swe_hweno_limit_f32": (I, [vp, dp, dp]),
        "swe_hweno_alpha_f32": (I, [vp, dp, ctypes.POINTER(D)]),
        "swe_hweno_step_f32": (I, [vp, dp, D, ctypes.POINTER(D)]),
        "swe_hweno_run_f32": (I, [vp, dp, I, D, ctypes.POINTER(D), ctypes.POINTER(I)]),
        "swe_hweno_rhs_vjp": (I, [vp, dp, D, D, dp, dp, dp, dp, dp]),
        "swe_hweno_limit_vjp": (I, [vp, dp, dp, dp, dp]),
        "swe_hweno_run_vjp": (I, [vp, dp, I, I, dp, dp, dp, dp, dp]),
        "swe_hweno_bottom_slopes": (I, [P, dp, dp, dp, vp]),
        "swe_hweno_run_checkpointed": (I, [vp, dp, I, I]),
        "swe_hweno_run_vjp_checkpointed": (I, [vp, I, I, dp, dp, dp, dp, dp]),
        "swe_hweno_bottom_slopes_vjp": (I, [P, dp, dp, dp, vp]),
        "swe_hweno_sync": (I, [vp]),
        "swe_hweno_destroy": (None, [vp]),
        "swe_hweno_strerror": (ctypes.c_char_p, [I]),
        "swe_hweno_abi_version": (I, []),
        "swe_hweno_tile": (I, [ctypes.POINTER(I), ctypes.POINTER(I)]),
        "swe_hweno_set_timing": (I, [vp, I]),
        "swe_hweno_ctx_tile": (I, [vp, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "swe_hweno_batch_init": (I, [P, ctypes.POINTER(Instance), I, vp, ctypes.POINTER(vp)]),
        "swe_hweno_batch_run": (I, [vp, I, ctypes.POINTER(D)]),
        "swe_hweno_batch_set_rows": (I, [vp, I]),
        "swe_hweno_batch_autotune": (I, [vp, ctypes.POINTER(I)]),
        "swe_hweno_batch_sync": (I, [vp]),
        "swe_hweno_batch_tune_cache_size": (I, []),
        "swe_hweno_batch_tune_cache_clear": (None, []),
        "swe_hweno_batch_destroy": (None, [vp]),
        "swe_hweno_get_timing": (I, [vp, ctypes.POINTER(D), ctypes.POINTER(ctypes.c_longlong)]),
        "swe_hweno_step_noalloc": (I, [P, dp, dp, dp, dp, D, vp, ctypes.POINTER(D)]),
        "swe_hweno_noalloc_capacity": (ctypes.c_ulong, []),
        "swe_hweno_math_check": (I, [I, dp, dp, ctypes.c_ulong, vp]),
        "swe_hweno_source_hash": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if L.swe_hweno_abi_version() != ABI_VERSION:
        raise ImportError("libswe_hweno.so ABI version mismatch; rebuild it")
    check_stamp(L)
    _lib = L
    return L


def check_stamp(L) -> str:
    """The library must have been built from the sources beside it (its stamp is the hash of the
    HIP sources, the header and the compile flags); a stale build is refused."""
    from .build import source_hash

    built = L.swe_hweno_source_hash().decode()
    want = source_hash()
    if built != want:
        raise ImportError(f"{LIB_PATH} was built from other sources (stamp {built}, sources {want}); "
                          "rebuild it with __graft_entry__.build()")
    return built


def strerror(code: int) -> str:
    try:
        return lib().swe_hweno_strerror(int(code)).decode()
    except ImportError:
        return f"error {code}"


def check(code: int, where: str = ""):
    if code != OK:
        raise SweError(code, where)
