"""The C ABI library builds, loads on a CPU-only host, exports every symbol the header declares,
and rejects bad arguments on the host before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2208_01260_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2208_01260_amd import build

        build.build()
    return _lib.lib()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "swe_hweno.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(swe_hweno_\w+)\s*\(", text)))


def test_exports_every_declared_symbol(L):
    from paper_2208_01260_amd import _lib

    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.EXPORTS) == names


def test_abi_version_and_messages(L):
    assert L.swe_hweno_abi_version() == 1
    assert L.swe_hweno_strerror(0) == b"ok"
    assert b"dry" in L.swe_hweno_strerror(-4)
    c, r = ctypes.c_int(), ctypes.c_int()
    assert L.swe_hweno_tile(ctypes.byref(c), ctypes.byref(r)) == 0 and c.value > 0 and r.value > 0


def _params(**kw):
    from paper_2208_01260_amd import _lib

    p = _lib.Params()
    d = dict(dim=2, nx=16, ny=16, x0=0.0, x1=1.0, y0=0.0, y1=1.0, g=9.812, cfl=0.6, eps=1e-6, bc_x=0, bc_y=0,
             flags=0, fixed_dt=0.0, alpha_x=0.0, alpha_y=0.0)
    d.update(kw)
    for k, v in d.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("bad", [
    dict(dim=3), dict(nx=3), dict(ny=2), dict(dim=1, ny=4), dict(x1=0.0), dict(y1=-1.0), dict(g=0.0),
    dict(cfl=-1.0), dict(eps=0.0), dict(eps=1e-21), dict(bc_x=2), dict(flags=64), dict(flags=1, fixed_dt=0.0),
    dict(flags=2, alpha_x=1.0, alpha_y=0.0), dict(g=float("nan")),
    dict(x1=float("inf")), dict(y0=float("-inf")), dict(x0=0.0, x1=1e-320),
    dict(flags=1, fixed_dt=float("inf")), dict(flags=2, alpha_x=float("inf"), alpha_y=1.0), dict(flags=16),
])
def test_init_rejects_bad_params_before_any_device_call(L, bad):
    p = _params(**bad)
    ctx = ctypes.c_void_p(123)
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert L.swe_hweno_init(ctypes.byref(p), fake, fake, fake, None, ctypes.byref(ctx)) == -1
    assert ctx.value is None
    ctx = ctypes.c_void_p(123)
    assert L.swe_hweno_init_f32(ctypes.byref(p), fake, fake, fake, None, ctypes.byref(ctx)) == -1
    assert ctx.value is None


def test_init_f32_rejects_eps_below_single_precision_floor(L):
    """The FP32 weights are of order eps^4 on flat data, so eps < 1e-9 is refused before any
    device call (eps = 1e-10 is valid for the FP64 context)."""
    p = _params(eps=1e-10)
    ctx = ctypes.c_void_p(123)
    fake = ctypes.c_void_p(0x1000)
    assert L.swe_hweno_init_f32(ctypes.byref(p), fake, fake, fake, None, ctypes.byref(ctx)) == -1
    assert ctx.value is None


def test_null_arguments_rejected(L):
    p = _params()
    ctx = ctypes.c_void_p()
    assert L.swe_hweno_init(None, None, None, None, None, ctypes.byref(ctx)) == -1
    assert L.swe_hweno_init(ctypes.byref(p), None, None, None, None, ctypes.byref(ctx)) == -1
    assert L.swe_hweno_init(ctypes.byref(p), ctypes.c_void_p(8), ctypes.c_void_p(8), None, None, ctypes.byref(ctx)) == -1
    assert L.swe_hweno_init(ctypes.byref(p), None, None, None, None, None) == -1
    assert L.swe_hweno_rhs(None, None, None, -1.0, -1.0) == -1
    assert L.swe_hweno_limit(None, None, None) == -1
    assert L.swe_hweno_step(None, None, 0.0, None) == -1
    assert L.swe_hweno_run(None, None, 1, 0.0, None, None) == -1
    assert L.swe_hweno_alpha(None, None, None) == -1
    assert L.swe_hweno_sync(None) == -1
    L.swe_hweno_destroy(None)  # no-op
    assert L.swe_hweno_tile(None, None) == -1
    assert L.swe_hweno_set_timing(None, 1) == -1
    assert L.swe_hweno_get_timing(None, None, None) == -1
    assert L.swe_hweno_ctx_tile(None, None, None) == -1
    assert L.swe_hweno_batch_run(None, 1, None) == -1
    assert L.swe_hweno_batch_set_rows(None, 8) == -1
    assert L.swe_hweno_batch_autotune(None, None) == -1
    assert L.swe_hweno_batch_sync(None) == -1
    L.swe_hweno_batch_tune_cache_clear()  # host-only
    assert L.swe_hweno_batch_tune_cache_size() == 0
    L.swe_hweno_batch_destroy(None)
    assert L.swe_hweno_init_f32(ctypes.byref(p), None, None, None, None, ctypes.byref(ctx)) == -1
    assert L.swe_hweno_rhs_f32(None, None, None, -1.0, -1.0) == -1
    assert L.swe_hweno_limit_f32(None, None, None) == -1
    assert L.swe_hweno_step_f32(None, None, 0.0, None) == -1
    assert L.swe_hweno_run_f32(None, None, 1, 0.0, None, None) == -1
    assert L.swe_hweno_alpha_f32(None, None, None) == -1
    assert L.swe_hweno_rhs_vjp(None, None, 1.0, 1.0, None, None, None, None, None) == -1
    assert L.swe_hweno_limit_vjp(None, None, None, None, None) == -1
    assert L.swe_hweno_run_vjp(None, None, 1, 1, None, None, None, None, None) == -1
    assert L.swe_hweno_run_checkpointed(None, None, 1, 1) == -1
    assert L.swe_hweno_run_vjp_checkpointed(None, 1, 1, None, None, None, None, None) == -1
    assert L.swe_hweno_bottom_slopes(None, None, None, None, None) == -1
    assert L.swe_hweno_bottom_slopes_vjp(None, None, None, None, None) == -1


def test_stale_library_is_refused(L, monkeypatch):
    """The binding checks the library's source stamp against the sources beside it: a library
    built from other sources fails to load (no silent use of a stale build)."""
    from paper_2208_01260_amd import _lib, build

    assert _lib.check_stamp(L) == build.source_hash()
    monkeypatch.setattr(build, "source_hash", lambda *a, **k: "0000000000000000")
    with pytest.raises(ImportError):
        _lib.check_stamp(L)


def test_math_check_validates_on_the_host(L):
    fake = ctypes.c_void_p(0x1000)
    assert L.swe_hweno_math_check(3, fake, fake, 4, None) == -1
    assert L.swe_hweno_math_check(-1, fake, fake, 4, None) == -1
    assert L.swe_hweno_math_check(0, None, fake, 4, None) == -1
    assert L.swe_hweno_math_check(0, fake, None, 4, None) == -1
    assert L.swe_hweno_math_check(0, fake, fake, 0, None) == -1


def test_noalloc_step_validates_on_the_host(L):
    """The allocation-free step checks its arguments and the size of its static array before any
    device call: null pointers, bad parameters and grids whose stage buffers exceed the array."""
    cap = L.swe_hweno_noalloc_capacity()
    assert cap == 32 << 20
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    ok = _params(nx=418, ny=418)
    assert 256 + 24 * 418 * 418 * 8 <= cap
    for p, args in ((None, (fake, fake, fake, fake)), (ok, (None, fake, fake, fake)), (ok, (fake, None, fake, fake)),
                    (ok, (fake, fake, None, fake)), (ok, (fake, fake, fake, None)),
                    (_params(nx=419, ny=418), (fake, fake, fake, fake)), (_params(dim=3), (fake, fake, fake, fake)),
                    (_params(dim=1, ny=1, nx=419431), (fake, fake, fake, None))):
        pp = ctypes.byref(p) if p is not None else None
        assert L.swe_hweno_step_noalloc(pp, *args, 0.0, None, None) == -1
    assert L.swe_hweno_step_noalloc(ctypes.byref(ok), fake, fake, fake, fake, float("nan"), None, None) == -1
    assert L.swe_hweno_step_noalloc(ctypes.byref(ok), fake, fake, fake, fake, float("inf"), None, None) == -1


def test_batch_init_rejects_bad_arguments(L):
    from paper_2208_01260_amd import _lib

    p = _params()
    arr = (_lib.Instance * 2)()
    for it in arr:
        it.nx, it.ny, it.x0, it.x1, it.y0, it.y1 = 16, 16, 0.0, 1.0, 0.0, 1.0
        it.b = it.bx = it.by = it.state = 0x1000  # never dereferenced: validation fails first
    h = ctypes.c_void_p(7)
    assert L.swe_hweno_batch_init(ctypes.byref(p), arr, 0, None, ctypes.byref(h)) == -1 and h.value is None
    arr[1].ny = 3
    assert L.swe_hweno_batch_init(ctypes.byref(p), arr, 2, None, ctypes.byref(h)) == -1
    arr[1].ny = 16
    arr[0].state = None
    assert L.swe_hweno_batch_init(ctypes.byref(p), arr, 2, None, ctypes.byref(h)) == -1
    p1 = _params(dim=1, ny=1)
    assert L.swe_hweno_batch_init(ctypes.byref(p1), arr, 2, None, ctypes.byref(h)) == -1


def test_product_path_has_no_cpu_fallback():
    """The Python front end only marshals arguments: it neither imports the oracle nor computes."""
    src = open(os.path.join(ROOT, "paper_2208_01260_amd", "solver.py")).read()
    src += open(os.path.join(ROOT, "paper_2208_01260_amd", "_lib.py")).read()
    assert "oracle" not in src
    assert "import numpy" not in src


def test_calibration_library_loads_and_checks_arguments():
    """The device calibration used by bench.py (sustained FP64 FMA stream) is built in-tree and
    rejects bad arguments on the host, before any device call."""
    from paper_2208_01260_amd import calib

    L = calib._load()
    t, m = ctypes.c_double(), ctypes.c_double()
    assert L.swe_calib_fp64_fma(3, 0.5, ctypes.byref(t), ctypes.byref(m)) == -1
    assert L.swe_calib_fp64_fma(16, 0.5, ctypes.byref(t), ctypes.byref(m)) == -1
    assert L.swe_calib_fp64_fma(2, 0.0, ctypes.byref(t), ctypes.byref(m)) == -1
    assert L.swe_calib_fp64_fma(2, 0.5, None, ctypes.byref(m)) == -1
