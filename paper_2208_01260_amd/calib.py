"""Device calibration for the stage kernels' roofline: the sustained FP64 FMA rate and shader
clock of a dense FMA stream (libswe_hweno_calib.so, built in-tree next to the solver library)."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libswe_hweno_calib.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        L.swe_calib_fp64_fma.restype = ctypes.c_int
        L.swe_calib_fp64_fma.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


def fp64_fma_ceiling(waves_per_simd=2, seconds=0.5):
    """(TFLOP/s, shader MHz) of a sustained FP64 FMA stream on the current device with
    waves_per_simd (1, 2, 4 or 8) wavefronts per SIMD, eight independent chains each."""
    t, m = ctypes.c_double(), ctypes.c_double()
    rc = _load().swe_calib_fp64_fma(int(waves_per_simd), float(seconds), ctypes.byref(t), ctypes.byref(m))
    if rc != 0:
        raise RuntimeError(f"swe_calib_fp64_fma failed ({rc})")
    return t.value, m.value
