"""TEST INFRASTRUCTURE — ctypes wrapper of the CPU oracle (``oracle/liboracle.so``).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package. It is a plain, slow, FP64 CPU implementation of the well-balanced
fifth-order finite-difference HWENO scheme for the shallow water equations (Zhao & Zhang 2022),
written from the paper and sharing no code with the HIP path.

Arrays are float64 numpy arrays. State layout: 1D ``(4, nx)`` = (eta, m, H, M); 2D ``(9, ny, nx)``
= (eta, m, w, H1, M1, W1, H2, M2, W2) with H1 = eta_x, ..., W2 = w_y. ``b``, ``bx`` (= b_x) and
``by`` (= b_y) are node planes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

FIXED_DT, FIXED_ALPHA, NO_LIMITER, LIMIT_BEFORE_RHS = 1, 2, 4, 8
PERIODIC, REFLECTIVE = 0, 1
ERRORS = {0: "ok", -1: "invalid argument", -4: "dry node (h <= 0)", -5: "non-finite value"}


class OracleError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double), ("y1", ctypes.c_double),
        ("g", ctypes.c_double), ("cfl", ctypes.c_double), ("eps", ctypes.c_double),
        ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int), ("flags", ctypes.c_int),
        ("fixed_dt", ctypes.c_double),
        ("alpha_x", ctypes.c_double * 3), ("alpha_y", ctypes.c_double * 3),
    ]


def build(force: bool = False) -> str:
    """Compile liboracle.so with make (g++ -O2 -ffp-contract=off -fopenmp)."""
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(["make", "-B" if force else "-s", "-C", _HERE, "liboracle.so"], check=True,
                       stdout=subprocess.DEVNULL)
    return _LIB_PATH


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(Params)
        I, Dd = ctypes.c_int, ctypes.c_double
        sig = {
            "orc_alpha": (I, [P, _D, _D, _D, _D, _D, _D]),
            "orc_rhs": (I, [P, _D, _D, _D, _D, Dd, Dd, _D]),
            "orc_limit": (I, [P, _D, _D, _D, _D, _D]),
            "orc_step": (I, [P, _D, _D, _D, _D, Dd, _D]),
            "orc_run": (I, [P, _D, _D, _D, _D, I, Dd, _D, ctypes.POINTER(I)]),
            "orc_run_delta_f32": (I, [P, _D, _D, _D, _D, I, Dd, _D, _D, ctypes.POINTER(I)]),
            "orc_rhs_f32": (I, [P, _D, _D, _D, _D, Dd, Dd, _D]),
            "orc_run_f32": (I, [P, _D, _D, _D, _D, I, Dd, _D, ctypes.POINTER(I)]),
            "orc_run_delta_f64": (I, [P, _D, _D, _D, _D, I, Dd, _D, _D, ctypes.POINTER(I)]),
            "orc_run_delta_f128": (I, [P, _D, _D, _D, _D, I, Dd, _D, _D, ctypes.POINTER(I)]),
            "orc_count_rhs": (I, [P, _D, _D, _D, _D, Dd, Dd, ctypes.POINTER(ctypes.c_longlong)]),
            "orc_count_limit": (I, [P, _D, _D, _D, _D, ctypes.POINTER(ctypes.c_longlong)]),
            "orc_rhs_jvp": (I, [P, _D, _D, _D, _D, _D, _D, _D, _D, Dd, Dd, _D, _D]),
            "orc_limit_jvp": (I, [P, _D, _D, _D, _D, _D, _D, _D, _D, _D, _D]),
            "orc_run_jvp": (I, [P, _D, _D, _D, _D, _D, _D, _D, _D, I, _D, _D]),
            "orc_hw_candidates": (None, [_D, _D, Dd, _D]),
            "orc_hw_beta": (None, [_D, _D, Dd, _D]),
            "orc_hw_weights": (None, [_D, Dd, _D]),
            "orc_hweno_value": (Dd, [_D, _D, Dd, Dd, _D]),
            "orc_hermite_dQ": (Dd, [_D, _D, Dd]),
            "orc_central4": (Dd, [Dd, Dd, Dd, Dd]),
            "orc_hweno_limit": (Dd, [Dd, Dd, Dd, Dd, Dd, Dd, Dd]),
            "orc_flux2d": (None, [I, _D, Dd, Dd, _D]),
            "orc_dflux2d": (None, [I, _D, Dd, _D, Dd, Dd, _D]),
            "orc_flux2d_tangent": (None, [I, _D, Dd, _D, Dd, Dd, _D]),
            "orc_eig2d": (None, [I, Dd, Dd, Dd, Dd, Dd, _D, _D]),
            "orc_flux1d": (None, [_D, Dd, Dd, _D]),
            "orc_dflux1d": (None, [_D, Dd, _D, Dd, Dd, _D]),
            "orc_flux1d_tangent": (None, [_D, Dd, _D, Dd, Dd, _D]),
            "orc_eig1d": (None, [Dd, Dd, Dd, Dd, _D, _D]),
            "orc_ssprk3_linear": (None, [Dd, Dd, Dd, I, _D, _D]),
            "orc_set_threads": (None, [I]),
            "orc_get_threads": (I, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a) -> ctypes.POINTER:
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _check(code: int):
    if code != 0:
        raise OracleError(ERRORS.get(code, f"error {code}"))


def make_params(dim, nx, ny=1, domain=(0.0, 1.0, 0.0, 1.0), g=9.812, cfl=0.6, eps=1e-6,
                bc=(PERIODIC, PERIODIC), flags=0, fixed_dt=0.0, alpha_x=(0, 0, 0), alpha_y=(0, 0, 0)) -> Params:
    p = Params()
    p.dim, p.nx, p.ny = dim, nx, (ny if dim == 2 else 1)
    p.x0, p.x1, p.y0, p.y1 = domain
    p.g, p.cfl, p.eps = g, cfl, eps
    p.bc_x, p.bc_y, p.flags = bc[0], bc[1], flags
    p.fixed_dt = fixed_dt
    for k in range(3):
        p.alpha_x[k] = alpha_x[k]
        p.alpha_y[k] = alpha_y[k]
    return p


def params_of(prob, **kw) -> Params:
    """Params for an inputs.Problem (any field can be overridden by keyword)."""
    d = dict(dim=prob.dim, nx=prob.nx, ny=prob.ny, domain=prob.domain, g=prob.g, cfl=prob.cfl,
             eps=prob.eps, bc=prob.bc)
    d.update(kw)
    return make_params(**d)


def set_threads(n: int):
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return lib().orc_get_threads()


def _bottom(p, b, bx, by):
    b, bx = _f64(b), _f64(bx)
    by = _f64(by) if p.dim == 2 else None
    return b, bx, by


def alpha(p, state, b, bx, by=None):
    state = _f64(state)
    b, bx, by = _bottom(p, b, bx, by)
    ax, ay = ctypes.c_double(), ctypes.c_double()
    _check(lib().orc_alpha(ctypes.byref(p), _p(state), _p(b), _p(bx), _p(by), ctypes.byref(ax), ctypes.byref(ay)))
    return ax.value, ay.value


def rhs(p, state, b, bx, by=None, alpha_x=-1.0, alpha_y=-1.0):
    state = _f64(state)
    b, bx, by = _bottom(p, b, bx, by)
    out = np.empty_like(state)
    _check(lib().orc_rhs(ctypes.byref(p), _p(state), _p(b), _p(bx), _p(by), alpha_x, alpha_y, _p(out)))
    return out


def rhs_f32(p, state, b, bx, by=None, alpha_x=-1.0, alpha_y=-1.0):
    """The right-hand side computed by the single-precision scheme (inputs rounded to float)."""
    state = _f64(state)
    b, bx, by = _bottom(p, b, bx, by)
    out = np.empty_like(state)
    _check(lib().orc_rhs_f32(ctypes.byref(p), _p(state), _p(b), _p(bx), _p(by), alpha_x, alpha_y, _p(out)))
    return out


def run_f32(p, state, b, bx, by=None, nsteps=0, t_end=0.0):
    """A run of the single-precision scheme; the final float state is returned widened."""
    s = np.array(state, dtype=np.float64, copy=True)
    b, bx, by = _bottom(p, b, bx, by)
    t, k = ctypes.c_double(), ctypes.c_int()
    _check(lib().orc_run_f32(ctypes.byref(p), _p(s), _p(b), _p(bx), _p(by), nsteps, t_end, ctypes.byref(t),
                             ctypes.byref(k)))
    return s, t.value, k.value


def limit(p, state, b, bx, by=None):
    state = _f64(state)
    b, bx, by = _bottom(p, b, bx, by)
    nd = 2 if p.dim == 1 else 6
    out = np.empty((nd,) + state.shape[1:], dtype=np.float64)
    _check(lib().orc_limit(ctypes.byref(p), _p(state), _p(b), _p(bx), _p(by), _p(out)))
    return out


def step(p, state, b, bx, by=None, dt=0.0):
    s = np.array(state, dtype=np.float64, copy=True)
    b, bx, by = _bottom(p, b, bx, by)
    used = ctypes.c_double()
    _check(lib().orc_step(ctypes.byref(p), _p(s), _p(b), _p(bx), _p(by), dt, ctypes.byref(used)))
    return s, used.value


def run(p, state, b, bx, by=None, nsteps=0, t_end=0.0):
    s = np.array(state, dtype=np.float64, copy=True)
    b, bx, by = _bottom(p, b, bx, by)
    t, k = ctypes.c_double(), ctypes.c_int()
    _check(lib().orc_run(ctypes.byref(p), _p(s), _p(b), _p(bx), _p(by), nsteps, t_end, ctypes.byref(t), ctypes.byref(k)))
    return s, t.value, k.value


def run_delta(precision, p, state, b, bx, by=None, nsteps=0, t_end=0.0):
    """Run in 'f32', 'f64' or 'f128' and return (final - initial) computed in that precision."""
    fn = {"f32": lib().orc_run_delta_f32, "f64": lib().orc_run_delta_f64, "f128": lib().orc_run_delta_f128}[precision]
    state = _f64(state)
    b, bx, by = _bottom(p, b, bx, by)
    delta = np.empty_like(state)
    t, k = ctypes.c_double(), ctypes.c_int()
    _check(fn(ctypes.byref(p), _p(state), _p(b), _p(bx), _p(by), nsteps, t_end, _p(delta), ctypes.byref(t), ctypes.byref(k)))
    return delta, t.value, k.value


def count_rhs(p, state, b, bx, by=None, alpha_x=1.0, alpha_y=1.0):
    """Arithmetic of one right-hand side: dict(add, mul, div, sqrt, cmp)."""
    state = _f64(state)
    b, bx, by = _bottom(p, b, bx, by)
    c = (ctypes.c_longlong * 5)()
    _check(lib().orc_count_rhs(ctypes.byref(p), _p(state), _p(b), _p(bx), _p(by), alpha_x, alpha_y, c))
    return dict(zip(("add", "mul", "div", "sqrt", "cmp"), list(c)))


def count_limit(p, state, b, bx, by=None):
    """Arithmetic of one limiter evaluation: dict(add, mul, div, sqrt, cmp)."""
    state = _f64(state)
    b, bx, by = _bottom(p, b, bx, by)
    c = (ctypes.c_longlong * 5)()
    _check(lib().orc_count_limit(ctypes.byref(p), _p(state), _p(b), _p(bx), _p(by), c))
    return dict(zip(("add", "mul", "div", "sqrt", "cmp"), list(c)))


def rhs_jvp(p, state, dstate, b, bx, by, db, dbx, dby, alpha_x, alpha_y):
    """Forward-mode tangent of the right-hand side (alpha frozen): returns (rhs, drhs)."""
    state, dstate = _f64(state), _f64(dstate)
    b, bx, by = _bottom(p, b, bx, by)
    db, dbx = _f64(db), _f64(dbx)
    dby = _f64(dby) if p.dim == 2 else None
    out, dout = np.empty_like(state), np.empty_like(state)
    _check(lib().orc_rhs_jvp(ctypes.byref(p), _p(state), _p(dstate), _p(b), _p(bx), _p(by), _p(db), _p(dbx),
                             _p(dby), alpha_x, alpha_y, _p(out), _p(dout)))
    return out, dout


def limit_jvp(p, state, dstate, b, bx, by, db, dbx, dby):
    """Forward-mode tangent of the limiter: returns (dmod, ddmod)."""
    state, dstate = _f64(state), _f64(dstate)
    b, bx, by = _bottom(p, b, bx, by)
    db, dbx = _f64(db), _f64(dbx)
    dby = _f64(dby) if p.dim == 2 else None
    nd = 2 if p.dim == 1 else 6
    out = np.empty((nd,) + state.shape[1:], dtype=np.float64)
    dout = np.empty_like(out)
    _check(lib().orc_limit_jvp(ctypes.byref(p), _p(state), _p(dstate), _p(b), _p(bx), _p(by), _p(db), _p(dbx),
                               _p(dby), _p(out), _p(dout)))
    return out, dout


def run_jvp(p, state, dstate, b, bx, by, db, dbx, dby, nsteps):
    """Forward-mode tangent of nsteps steps (use FIXED_DT | FIXED_ALPHA for a smooth map):
    returns (final state, its directional derivative)."""
    state, dstate = _f64(state), _f64(dstate)
    b, bx, by = _bottom(p, b, bx, by)
    db, dbx = _f64(db), _f64(dbx)
    dby = _f64(dby) if p.dim == 2 else None
    out, dout = np.empty_like(state), np.empty_like(state)
    _check(lib().orc_run_jvp(ctypes.byref(p), _p(state), _p(dstate), _p(b), _p(bx), _p(by), _p(db), _p(dbx),
                             _p(dby), int(nsteps), _p(out), _p(dout)))
    return out, dout


# ----------------------------------------------------------------- building blocks (for pins)
def _vec(x, n=3):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(n))


def hw_candidates(f, p, dx):
    q = np.empty(3)
    lib().orc_hw_candidates(_p(_vec(f)), _p(_vec(p)), dx, _p(q))
    return q


def hw_beta(f, p, dx):
    q = np.empty(3)
    lib().orc_hw_beta(_p(_vec(f)), _p(_vec(p)), dx, _p(q))
    return q


def hw_weights(beta, eps):
    w = np.empty(3)
    lib().orc_hw_weights(_p(_vec(beta)), eps, _p(w))
    return w


def hweno_value(f, p, dx, eps):
    w = np.empty(3)
    v = lib().orc_hweno_value(_p(_vec(f)), _p(_vec(p)), dx, eps, _p(w))
    return v, w


def hermite_dQ(f, p, dx):
    return lib().orc_hermite_dQ(_p(_vec(f)), _p(_vec(p)), dx)


def central4(a, b, c, d):
    return lib().orc_central4(a, b, c, d)


def hweno_limit(mm, m0, mp, nm, np_, dx, eps):
    return lib().orc_hweno_limit(mm, m0, mp, nm, np_, dx, eps)


def flux2d(direction, U, b, g=9.812):
    F = np.empty(3)
    lib().orc_flux2d(direction, _p(_vec(U)), b, g, _p(F))
    return F


def dflux2d(direction, U, b, D, B, g=9.812):
    P = np.empty(3)
    lib().orc_dflux2d(direction, _p(_vec(U)), b, _p(_vec(D)), B, g, _p(P))
    return P


def flux2d_tangent(direction, U, b, dU, db, g=9.812):
    F = np.empty(3)
    lib().orc_flux2d_tangent(direction, _p(_vec(U)), b, _p(_vec(dU)), db, g, _p(F))
    return F


def eig2d(direction, eta, m, w, b, g=9.812):
    L, R = np.empty(9), np.empty(9)
    lib().orc_eig2d(direction, eta, m, w, b, g, _p(L), _p(R))
    return L.reshape(3, 3), R.reshape(3, 3)


def flux1d(U, b, g=9.812):
    F = np.empty(2)
    lib().orc_flux1d(_p(_vec(U, 2)), b, g, _p(F))
    return F


def dflux1d(U, b, V, B, g=9.812):
    P = np.empty(2)
    lib().orc_dflux1d(_p(_vec(U, 2)), b, _p(_vec(V, 2)), B, g, _p(P))
    return P


def flux1d_tangent(U, b, dU, db, g=9.812):
    F = np.empty(2)
    lib().orc_flux1d_tangent(_p(_vec(U, 2)), b, _p(_vec(dU, 2)), db, g, _p(F))
    return F


def eig1d(eta, m, b, g=9.812):
    L, R = np.empty(4), np.empty(4)
    lib().orc_eig1d(eta, m, b, g, _p(L), _p(R))
    return L.reshape(2, 2), R.reshape(2, 2)


def ssprk3_linear(lam, mu, dt, u0, d0, lim_first=False):
    U, D = np.array([u0], dtype=np.float64), np.array([d0], dtype=np.float64)
    lib().orc_ssprk3_linear(lam, mu, dt, int(lim_first), _p(U), _p(D))
    return U[0], D[0]
