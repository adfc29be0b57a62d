"""Seeded synthetic inputs for the HWENO shallow-water solver.

This module holds no arithmetic of the numerical method. It only samples bottoms and initial
states (with their analytic derivatives, obtained by complex-step differentiation of the
closed-form initial data) and packs them as float64 arrays in the paper's variables:

* 1D state ``(4, nx)``: eta = h + b, m = hu, H = eta_x, M = m_x
* 2D state ``(9, ny, nx)``: eta, m = hu, w = hv, (H1, M1, W1) = U_x, (H2, M2, W2) = U_y
* bottom ``b``, ``bx`` = b_x, ``by`` = b_y (2D)

Nodes sit at cell centres, x_i = x0 + (i + 1/2) dx. Derivatives of piecewise-constant data
(a dam-break interface, a strip perturbation, a step bottom) are zero, the delta ignored.

Workloads (seed = 220801260 + workload index):

1. ``c1_1d``        1D, N = 200, periodic [0, 1]; bottom = 3 seeded Fourier modes (total
                    amplitude <= 0.3); eta = 2 plus a seeded periodic Gaussian bump of 1e-3.
2. ``c2_2d``        2D, 400^2, [0, 2]^2, reflective; bottom = 4 seeded Gaussian bumps
                    (amplitude 0.3-0.8, width 0.05-0.2); eta = 1 plus 0.01 in 0.05 < x < 0.15
                    (``variant='smooth'`` replaces the strip by a Gaussian; ``'rest'`` drops it;
                    ``'flat'`` sets b = 0).
3. ``c3_2d``        2D, 4096^2, [0, 1]^2, reflective, dam break: eta = 10 left of a
                    random-phase sinusoidal interface near x = 0.5, 5 right of it; bottom = 4
                    seeded Gaussian bumps (amplitude 0.5-2).
4. ``c4_batch``     256 instances with sizes drawn from {64, 96, ..., 512}^2, own bottoms
                    (2-6 bumps) and small perturbations.
5. ``c5_adjoint``   256^2 lake at rest plus a perturbation, a target bottom and gauge nodes.

Paper problems (Sec. 4): ``paper_accuracy_1d`` (Ex. 4.1), ``paper_lake_1d`` (Ex. 4.2, smooth and
step bottoms), ``paper_perturbed_1d`` (Ex. 4.3), ``paper_accuracy_2d`` (Ex. 4.6),
``paper_lake_2d`` (Ex. 4.7), ``paper_perturbed_2d`` (Ex. 4.8), ``paper_dam_2d`` (Ex. 4.9).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 220801260
G = 9.812
PERIODIC, REFLECTIVE = 0, 1


@dataclass
class Problem:
    name: str
    dim: int
    nx: int
    ny: int
    domain: tuple
    bc: tuple
    state: np.ndarray
    b: np.ndarray
    bx: np.ndarray
    by: np.ndarray | None
    g: float = G
    cfl: float = 0.6
    eps: float = 1e-6
    t_end: float = 0.0
    nsteps: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def dx(self):
        return (self.domain[1] - self.domain[0]) / self.nx

    @property
    def dy(self):
        return (self.domain[3] - self.domain[2]) / self.ny if self.dim == 2 else 1.0

    @property
    def cells(self):
        return self.nx * (self.ny if self.dim == 2 else 1)


# ------------------------------------------------------------------ grids and derivatives
def nodes_1d(n, x0, x1):
    dx = (x1 - x0) / n
    return x0 + (np.arange(n) + 0.5) * dx


def nodes_2d(nx, ny, domain):
    x = nodes_1d(nx, domain[0], domain[1])
    y = nodes_1d(ny, domain[2], domain[3])
    return np.meshgrid(x, y, indexing="xy")  # arrays (ny, nx)


_H = 1e-30


def d_dx(f, x, *rest):
    """Exact-to-round-off derivative of an analytic numpy expression by the complex step."""
    return np.imag(f(x + 1j * _H, *rest)) / _H


def d_dy(f, x, y):
    return np.imag(f(x, y + 1j * _H)) / _H


def real(f, *args):
    return np.real(f(*args)).astype(np.float64)


def _mk1d(name, n, dom, bc, bfun, etafun, mfun, **kw):
    x = nodes_1d(n, dom[0], dom[1])
    b, bx = real(bfun, x), d_dx(bfun, x)
    st = np.stack([real(etafun, x), real(mfun, x), d_dx(etafun, x), d_dx(mfun, x)])
    return Problem(name, 1, n, 1, (dom[0], dom[1], 0.0, 1.0), (bc, PERIODIC), np.ascontiguousarray(st),
                   b, bx, None, **kw)


def _mk2d(name, nx, ny, dom, bc, bfun, etafun, mfun, wfun, **kw):
    X, Y = nodes_2d(nx, ny, dom)
    b, bx, by = real(bfun, X, Y), d_dx(bfun, X, Y), d_dy(bfun, X, Y)
    f = (etafun, mfun, wfun)
    st = [real(fn, X, Y) for fn in f] + [d_dx(fn, X, Y) for fn in f] + [d_dy(fn, X, Y) for fn in f]
    return Problem(name, 2, nx, ny, tuple(dom), tuple(bc), np.ascontiguousarray(np.stack(st)), b, bx, by, **kw)


def _zero(x, *rest):
    return 0.0 * x


def _gaussians(rng, nb, amp, sig, lo, hi, maxb, dom, nx_probe=256):
    """Sum of seeded Gaussian bumps a exp(-r^2 / (2 s^2)), rejected until max b <= maxb."""
    X, Y = nodes_2d(nx_probe, nx_probe, dom)
    while True:
        a = rng.uniform(*amp, size=nb)
        s = rng.uniform(*sig, size=nb)
        cx = rng.uniform(lo, hi, size=nb)
        cy = rng.uniform(lo, hi, size=nb)

        def bfun(x, y, a=a, s=s, cx=cx, cy=cy):
            out = 0.0 * x
            for k in range(len(a)):
                out = out + a[k] * np.exp(-((x - cx[k]) ** 2 + (y - cy[k]) ** 2) / (2 * s[k] ** 2))
            return out

        if np.max(real(bfun, X, Y)) <= maxb:
            return bfun, dict(a=a, s=s, cx=cx, cy=cy)


# ------------------------------------------------------------------ workloads
def c1_1d(n=200, rest=False, eps=1e-6, seed=None):
    rng = np.random.default_rng(SEED_BASE + 1 if seed is None else seed)
    modes = rng.choice(np.arange(1, 5), size=3, replace=False)
    amps = rng.uniform(0.05, 0.1, size=3)
    phs = rng.uniform(0, 2 * np.pi, size=3)
    kappa = rng.uniform(20, 60)
    xc = rng.uniform(0.3, 0.7)

    def bfun(x):
        return sum(amps[k] * np.sin(2 * np.pi * modes[k] * x + phs[k]) for k in range(3))

    def eta(x):
        if rest:
            return 2.0 + 0.0 * x
        return 2.0 + 1e-3 * np.exp(kappa * (np.cos(2 * np.pi * (x - xc)) - 1.0))

    return _mk1d("c1_1d_rest" if rest else "c1_1d", n, (0.0, 1.0), PERIODIC, bfun, eta, _zero,
                 eps=eps, t_end=0.1)


def c2_2d(n=400, variant="strip", seed=None, ny=None):
    ny = n if ny is None else ny
    rng = np.random.default_rng(SEED_BASE + 2 if seed is None else seed)
    dom = (0.0, 2.0, 0.0, 2.0)
    if variant == "flat":
        bfun = _zero2
    else:
        bfun, _ = _gaussians(rng, 4, (0.3, 0.8), (0.05, 0.2), 0.4, 1.6, 0.9, dom)

    def eta(x, y):
        if variant == "strip":
            return 1.0 + 0.01 * ((x.real > 0.05) & (x.real < 0.15)) + 0.0 * x
        if variant in ("smooth", "flat"):
            return 1.0 + 0.01 * np.exp(-((x - 0.1) ** 2) / (2 * 0.02 ** 2)) + 0.0 * y
        return 1.0 + 0.0 * x

    return _mk2d(f"c2_2d_{variant}", n, ny, dom, (REFLECTIVE, REFLECTIVE), bfun, eta, _zero2, _zero2,
                 nsteps=200)


def _zero2(x, y):
    return 0.0 * x + 0.0 * y


def c3_2d(n=4096, seed=None, ny=None):
    ny = n if ny is None else ny
    rng = np.random.default_rng(SEED_BASE + 3 if seed is None else seed)
    dom = (0.0, 1.0, 0.0, 1.0)
    bfun, _ = _gaussians(rng, 4, (0.5, 2.0), (0.05, 0.15), 0.1, 0.9, 4.0, dom)
    ph = rng.uniform(0, 2 * np.pi, size=3)

    def eta(x, y):
        xi = 0.5 + 0.02 * sum(np.sin(2 * np.pi * k * y.real + ph[k - 1]) / k for k in (1, 2, 3))
        return np.where(x.real < xi, 10.0, 5.0) + 0.0 * x

    return _mk2d("c3_2d", n, ny, dom, (REFLECTIVE, REFLECTIVE), bfun, eta, _zero2, _zero2, nsteps=50)


def c4_instance(rng, sizes=tuple(range(64, 513, 32))):
    nx = int(rng.choice(sizes))
    ny = int(rng.choice(sizes))
    dom = (0.0, 2.0, 0.0, 2.0)
    nb = int(rng.integers(2, 7))
    bfun, _ = _gaussians(rng, nb, (0.3, 0.8), (0.05, 0.2), 0.4, 1.6, 0.9, dom, nx_probe=128)
    cx, cy = rng.uniform(0.3, 1.7, size=2)

    def eta(x, y):
        return 1.0 + 0.01 * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * 0.05 ** 2))

    return _mk2d("c4_instance", nx, ny, dom, (REFLECTIVE, REFLECTIVE), bfun, eta, _zero2, _zero2, nsteps=100)


def c4_batch(count=256, seed=None):
    rng = np.random.default_rng(SEED_BASE + 4 if seed is None else seed)
    return [c4_instance(rng) for _ in range(count)]


def c5_adjoint(n=256, seed=None):
    rng = np.random.default_rng(SEED_BASE + 5 if seed is None else seed)
    dom = (0.0, 2.0, 0.0, 2.0)
    bfun, _ = _gaussians(rng, 4, (0.3, 0.8), (0.05, 0.2), 0.4, 1.6, 0.9, dom)
    cx, cy = rng.uniform(0.5, 1.5, size=2)

    def eta(x, y):
        return 1.0 + 0.01 * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * 0.05 ** 2))

    prob = _mk2d("c5_adjoint", n, n, dom, (REFLECTIVE, REFLECTIVE), bfun, eta, _zero2, _zero2, nsteps=100)
    dcx, dcy = rng.uniform(0.5, 1.5, size=2)

    def dbfun(x, y):
        return 0.05 * np.exp(-((x - dcx) ** 2 + (y - dcy) ** 2) / (2 * 0.1 ** 2))

    X, Y = nodes_2d(n, n, dom)
    prob.extra["target_db"] = real(dbfun, X, Y)
    prob.extra["target_dbx"] = d_dx(dbfun, X, Y)
    prob.extra["target_dby"] = d_dy(dbfun, X, Y)
    gi = rng.integers(10, n - 10, size=16)
    gj = rng.integers(10, n - 10, size=16)
    prob.extra["gauges"] = np.stack([gj, gi], axis=1)
    return prob


# ------------------------------------------------------------------ the paper's problems (Sec. 4)
def paper_accuracy_1d(n):
    """Ex. 4.1: b = sin^2(pi x), h = 5 + exp(cos 2 pi x), hu = sin(cos 2 pi x), periodic, t = 0.1."""
    def bfun(x):
        return np.sin(np.pi * x) ** 2

    def eta(x):
        return 5.0 + np.exp(np.cos(2 * np.pi * x)) + bfun(x)

    def m(x):
        return np.sin(np.cos(2 * np.pi * x))

    return _mk1d("paper_accuracy_1d", n, (0.0, 1.0), PERIODIC, bfun, eta, m, t_end=0.1)


def paper_lake_1d(kind="smooth", n=200):
    """Ex. 4.2: lake at rest h + b = 10 over b = 5 exp(-2/5 (x-5)^2) or a step of 4 on [4, 8]."""
    if kind == "smooth":
        def bfun(x):
            return 5.0 * np.exp(-0.4 * (x - 5.0) ** 2)
    else:
        def bfun(x):
            return np.where((x.real >= 4.0) & (x.real <= 8.0), 4.0, 0.0) + 0.0 * x

    def eta(x):
        return 10.0 + 0.0 * x

    return _mk1d(f"paper_lake_1d_{kind}", n, (0.0, 10.0), PERIODIC, bfun, eta, _zero, t_end=0.5)


def paper_perturbed_1d(pulse=0.2, n=200):
    """Ex. 4.3: bump b on [1.4, 1.6], h = 1 - b (+ pulse on [1.1, 1.2]), u = 0, t = 0.2."""
    def bfun(x):
        xr = x.real
        return np.where((xr >= 1.4) & (xr <= 1.6), 0.25 * (np.cos(10 * np.pi * (x - 1.5)) + 1.0), 0.0 * x)

    def eta(x):
        xr = x.real
        return 1.0 + np.where((xr >= 1.1) & (xr <= 1.2), pulse, 0.0) + 0.0 * x

    return _mk1d("paper_perturbed_1d", n, (0.0, 2.0), REFLECTIVE, bfun, eta, _zero, t_end=0.2,
                 eps=1e-10 if pulse < 0.01 else 1e-6)


def paper_wavy_1d(n=200):
    """Ex. 4.4: wavy bottom b = 0.3 cos^30(pi/2 (x-1)) on [0, 2] (0 elsewhere) in [-10, 10];
    h + b = 2, u = 1 for x <= 1 and h + b = 0.35, u = 0 beyond; t = 1. The paper states no
    boundary condition: reflective walls here (no wave reaches the region the paper plots by t = 1)."""
    def bfun(x):
        xr = x.real
        return np.where((xr >= 0.0) & (xr <= 2.0), 0.3 * np.cos(0.5 * np.pi * (x - 1.0)) ** 30, 0.0 * x)

    def eta(x):
        return np.where(x.real <= 1.0, 2.0, 0.35) + 0.0 * x

    def m(x):
        return np.where(x.real <= 1.0, 2.0 - bfun(x), 0.0 * x)

    return _mk1d("paper_wavy_1d", n, (-10.0, 10.0), REFLECTIVE, bfun, eta, m, t_end=1.0)


def paper_rect_dam_1d(n=200, t_end=15.0):
    """Ex. 4.5: dam break over a rectangular hump b = 8 on |x - 750| <= 1500/8 in (0, 1500);
    h + b = 20 for x <= 750, 15 beyond, u = 0; t = 15 and 60. Reflective walls (the paper states
    none; by t = 15 no wave has reached them)."""
    def bfun(x):
        return np.where(np.abs(x.real - 750.0) <= 1500.0 / 8.0, 8.0, 0.0) + 0.0 * x

    def eta(x):
        return np.where(x.real <= 750.0, 20.0, 15.0) + 0.0 * x

    return _mk1d("paper_rect_dam_1d", n, (0.0, 1500.0), REFLECTIVE, bfun, eta, _zero, t_end=t_end)


def paper_accuracy_2d(n):
    """Ex. 4.6: b = sin 2 pi x + sin 2 pi y, periodic on [0,1]^2, t = 0.05."""
    def bfun(x, y):
        return np.sin(2 * np.pi * x) + np.sin(2 * np.pi * y)

    def eta(x, y):
        return 10.0 + np.exp(np.sin(2 * np.pi * x)) * np.cos(2 * np.pi * y) + bfun(x, y)

    def m(x, y):
        return np.sin(np.cos(2 * np.pi * x)) * np.sin(2 * np.pi * y)

    def w(x, y):
        return np.cos(2 * np.pi * x) * np.cos(np.sin(2 * np.pi * y))

    return _mk2d("paper_accuracy_2d", n, n, (0.0, 1.0, 0.0, 1.0), (PERIODIC, PERIODIC), bfun, eta, m, w,
                 t_end=0.05)


def paper_lake_2d(n=200):
    """Ex. 4.7: lake at rest h + b = 1 over b = 0.8 exp(-50 r^2), periodic on [0,1]^2, t = 0.1."""
    def bfun(x, y):
        return 0.8 * np.exp(-50.0 * ((x - 0.5) ** 2 + (y - 0.5) ** 2))

    def eta(x, y):
        return 1.0 + 0.0 * x

    return _mk2d("paper_lake_2d", n, n, (0.0, 1.0, 0.0, 1.0), (PERIODIC, PERIODIC), bfun, eta, _zero2, _zero2,
                 t_end=0.1)


def paper_perturbed_2d(nx=200, ny=100, pad=0.0):
    """Ex. 4.8: b = 0.8 exp(-5(x-0.9)^2 - 50(y-0.5)^2) on [0,2]x[0,1], h = 1 - b (+0.01 on 0.05<x<0.15).

    The paper gives no boundary condition; its comparison ranges are those of a run whose waves
    leave the domain. pad > 0 extends the domain by pad on both sides in x (same dx, reflective
    walls farther out) so that the walls' reflections re-enter [0, 2] only after t = 2 pad / sqrt(g);
    extra["window_x"] is the paper's x-range."""
    dx = 2.0 / nx
    extra = int(round(pad / dx))
    dom = (-extra * dx, 2.0 + extra * dx, 0.0, 1.0)

    def bfun(x, y):
        return 0.8 * np.exp(-5.0 * (x - 0.9) ** 2 - 50.0 * (y - 0.5) ** 2)

    def eta(x, y):
        xr = x.real
        return 1.0 + np.where((xr >= 0.05) & (xr <= 0.15), 0.01, 0.0) + 0.0 * x

    pr = _mk2d("paper_perturbed_2d", nx + 2 * extra, ny, dom, (REFLECTIVE, REFLECTIVE), bfun, eta,
               _zero2, _zero2, t_end=0.12)
    pr.extra["window_x"] = (0.0, 2.0)
    return pr


def paper_dam_2d(n=200):
    """Ex. 4.9: circular dam break over a bump on [0,2]^2, t = 0.15."""
    def bfun(x, y):
        r = np.sqrt((x.real - 1.5) ** 2 + (y.real - 1.0) ** 2)
        return np.where(r <= 0.5, 0.125 * (np.cos(2 * np.pi * (x - 0.5)) + 1.0) * (np.cos(2 * np.pi * y) + 1.0),
                        0.0 * x)

    def eta(x, y):
        r = np.sqrt((x.real - 1.25) ** 2 + (y.real - 1.0) ** 2)
        return np.where(r <= 0.1, 1.1, 0.6) + 0.0 * x

    return _mk2d("paper_dam_2d", n, n, (0.0, 2.0, 0.0, 2.0), (REFLECTIVE, REFLECTIVE), bfun, eta, _zero2, _zero2,
                 t_end=0.15)
