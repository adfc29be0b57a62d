"""Pins of the oracle's building blocks against definitions that are independent of its code.

Each reconstruction formula printed in the paper (Sec. 2.1, 2.2, eq. (3.7)) is the value of a
polynomial defined by interpolation conditions. Here the polynomials are built from those
conditions with numpy (a linear solve) and the oracle's closed forms must reproduce them:
  * q1, q2, q3 and Q' are exact for cell averages of cubics / quintics;
  * beta_l is the Jiang-Shu indicator sum_k dx^(2k-1) int_{I_i} (q_l^(k))^2 of the fitted cubic;
  * with eps -> infinity the weights become gamma and F^ equals the quintic Hermite value Q;
  * the limiter's p'_l and beta^L_l follow from the quadratic Hermite interpolants;
  * the four-point mixed flux reproduces a cubic from its cell averages;
  * the flux Jacobians and eigenvectors agree with forward-mode derivatives of the printed
    fluxes (L R = I, L J R = diag(lambda)).
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as Pn

RNG = np.random.default_rng(12345)


def cell_avg(c, k, dx):
    """Average of the polynomial c(x) over the cell [ (k-1/2) dx, (k+1/2) dx ]."""
    ci = Pn.polyint(c)
    return (Pn.polyval((k + 0.5) * dx, ci) - Pn.polyval((k - 0.5) * dx, ci)) / dx


def dcell_avg(c, k, dx):
    return (Pn.polyval((k + 0.5) * dx, c) - Pn.polyval((k - 0.5) * dx, c)) / dx


def hermite_fit(cells_f, cells_p, f, p, dx):
    deg = len(cells_f) + len(cells_p) - 1
    A, rhs = [], []
    for k in cells_f:
        A.append([cell_avg(np.eye(deg + 1)[m], k, dx) for m in range(deg + 1)])
        rhs.append(f[k + 1])
    for k in cells_p:
        A.append([dcell_avg(np.eye(deg + 1)[m], k, dx) for m in range(deg + 1)])
        rhs.append(p[k + 1])
    return np.linalg.solve(np.array(A), np.array(rhs))


def js_indicator(c, dx, order):
    s = 0.0
    for k in range(1, order + 1):
        d = Pn.polyder(c, k)
        di = Pn.polyint(Pn.polymul(d, d))
        s += dx ** (2 * k - 1) * (Pn.polyval(0.5 * dx, di) - Pn.polyval(-0.5 * dx, di))
    return s


@pytest.mark.parametrize("dx", [1.0, 0.37, 0.013])
def test_candidates_and_beta_match_hermite_definitions(oracle_mod, dx):
    O = oracle_mod
    for _ in range(5):
        f, p = RNG.normal(size=3), RNG.normal(size=3) / dx
        q1 = hermite_fit([-1, 0], [-1, 0], f, p, dx)
        q2 = hermite_fit([0, 1], [0, 1], f, p, dx)
        q3 = hermite_fit([-1, 0, 1], [0], f, p, dx)
        Q = hermite_fit([-1, 0, 1], [-1, 0, 1], f, p, dx)
        want_q = [Pn.polyval(0.5 * dx, c) for c in (q1, q2, q3)]
        np.testing.assert_allclose(O.hw_candidates(f, p, dx), want_q, rtol=1e-11, atol=1e-11)
        want_b = [js_indicator(c, dx, 3) for c in (q1, q2, q3)]
        np.testing.assert_allclose(O.hw_beta(f, p, dx), want_b, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(O.hermite_dQ(f, p, dx), Pn.polyval(0.5 * dx, Pn.polyder(Q)), rtol=1e-10,
                                   atol=1e-10 / dx)
        # linear weights gamma reproduce the quintic: eps -> infinity
        v, w = O.hweno_value(f, p, dx, 1e30)
        np.testing.assert_allclose(w, [0.3, 0.3, 0.4], rtol=1e-14)
        np.testing.assert_allclose(v, Pn.polyval(0.5 * dx, Q), rtol=1e-11, atol=1e-11)


def test_candidates_exact_for_cubic_cell_averages(oracle_mod):
    O = oracle_mod
    dx = 0.05
    for _ in range(5):
        c = RNG.normal(size=4)
        f = np.array([cell_avg(c, k, dx) for k in (-1, 0, 1)])
        p = np.array([dcell_avg(c, k, dx) for k in (-1, 0, 1)])
        np.testing.assert_allclose(O.hw_candidates(f, p, dx), [Pn.polyval(0.5 * dx, c)] * 3, rtol=1e-12, atol=1e-12)
        c5 = RNG.normal(size=6)
        f = np.array([cell_avg(c5, k, dx) for k in (-1, 0, 1)])
        p = np.array([dcell_avg(c5, k, dx) for k in (-1, 0, 1)])
        np.testing.assert_allclose(O.hermite_dQ(f, p, dx), Pn.polyval(0.5 * dx, Pn.polyder(c5)), rtol=1e-10)


def test_weights_definition_and_eno_property(oracle_mod):
    O = oracle_mod
    be = np.array([1e-3, 2.0, 0.5])
    eps = 1e-6
    wt = np.array([0.3, 0.3, 0.4]) / (be + eps) ** 2
    np.testing.assert_allclose(O.hw_weights(be, eps), wt / wt.sum(), rtol=1e-14)
    # a jump between x_i and x_{i+1}: only q1 (cells i-1, i) is smooth
    v, w = O.hweno_value([1.0, 1.0, 0.0], [0.0, 0.0, 0.0], 0.01, 1e-6)
    assert w[0] > 0.999999 and abs(v - 1.0) < 1e-6


def test_limiter_matches_quadratic_hermite_definitions(oracle_mod):
    O = oracle_mod
    dx = 0.21
    for _ in range(5):
        mu = RNG.normal(size=3)
        nu = RNG.normal(size=2)
        # p1: p(x_{i-1}) = mu_-1, p(x_i) = mu_0, p'(x_{i-1}) = nu_-1; p2 mirrored; p3 through 3 points
        def fit(conds):
            A = [[(x ** m if kind == "v" else (m * x ** (m - 1) if m else 0.0)) for m in range(3)] for kind, x, _ in conds]
            return np.linalg.solve(np.array(A), np.array([v for _, _, v in conds]))
        p1 = fit([("v", -dx, mu[0]), ("v", 0.0, mu[1]), ("d", -dx, nu[0])])
        p2 = fit([("v", 0.0, mu[1]), ("v", dx, mu[2]), ("d", dx, nu[1])])
        p3 = fit([("v", -dx, mu[0]), ("v", 0.0, mu[1]), ("v", dx, mu[2])])
        dp = np.array([Pn.polyval(0.0, Pn.polyder(c)) for c in (p1, p2, p3)])
        be = np.array([js_indicator(c, dx, 2) for c in (p1, p2, p3)])
        eps = 1e-6
        wt = np.array([0.25, 0.25, 0.5]) / (be + eps) ** 2
        want = np.dot(wt / wt.sum(), dp)
        got = O.hweno_limit(mu[0], mu[1], mu[2], nu[0], nu[1], dx, eps)
        np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12)
        # linear weights (1/4, 1/4, 1/2)
        got = O.hweno_limit(mu[0], mu[1], mu[2], nu[0], nu[1], dx, 1e30)
        np.testing.assert_allclose(got, np.dot([0.25, 0.25, 0.5], dp), rtol=1e-10, atol=1e-12)


def test_limiter_keeps_exact_derivative_of_quadratics(oracle_mod):
    O = oracle_mod
    dx = 0.1
    c = RNG.normal(size=3)
    mu = [Pn.polyval(x, c) for x in (-dx, 0.0, dx)]
    nu = [Pn.polyval(x, Pn.polyder(c)) for x in (-dx, dx)]
    got = O.hweno_limit(mu[0], mu[1], mu[2], nu[0], nu[1], dx, 1e-6)
    np.testing.assert_allclose(got, Pn.polyval(0.0, Pn.polyder(c)), rtol=1e-12, atol=1e-12)


def test_central4_reproduces_cubic_from_cell_averages(oracle_mod):
    O = oracle_mod
    dx = 0.3
    c = RNG.normal(size=4)
    a = [cell_avg(c, k, dx) for k in (-1, 0, 1, 2)]
    np.testing.assert_allclose(O.central4(*a), Pn.polyval(0.5 * dx, c), rtol=1e-12)


@pytest.mark.parametrize("direction", [0, 1])
def test_jacobian_and_eigenvectors_2d(oracle_mod, direction):
    O = oracle_mod
    g = 9.812
    for _ in range(5):
        b = RNG.uniform(-1, 1)
        U = np.array([b + RNG.uniform(0.5, 3.0), RNG.normal(), RNG.normal()])
        D, B = RNG.normal(size=3), RNG.normal()
        # derivative flux = forward-mode derivative of the printed flux along (D, B)
        np.testing.assert_allclose(O.dflux2d(direction, U, b, D, B, g), O.flux2d_tangent(direction, U, b, D, B, g),
                                   rtol=1e-13, atol=1e-13)
        J = np.stack([O.flux2d_tangent(direction, U, b, e, 0.0, g) for e in np.eye(3)], axis=1)
        L, R = O.eig2d(direction, U[0], U[1], U[2], b, g)
        np.testing.assert_allclose(L @ R, np.eye(3), atol=1e-13)
        h = U[0] - b
        un = (U[1] if direction == 0 else U[2]) / h
        c = np.sqrt(g * h)
        np.testing.assert_allclose(L @ J @ R, np.diag([un - c, un, un + c]), atol=1e-12)
        # the middle characteristic row annihilates the bottom vector (0,b,0) / (0,0,b)
        assert L[1, 1 + direction] == 0.0


def test_jacobian_and_eigenvectors_1d(oracle_mod):
    O = oracle_mod
    g = 9.812
    for _ in range(5):
        b = RNG.uniform(-1, 1)
        U = np.array([b + RNG.uniform(0.5, 3.0), RNG.normal()])
        V, B = RNG.normal(size=2), RNG.normal()
        np.testing.assert_allclose(O.dflux1d(U, b, V, B, g), O.flux1d_tangent(U, b, V, B, g), rtol=1e-13, atol=1e-13)
        J = np.stack([O.flux1d_tangent(U, b, e, 0.0, g) for e in np.eye(2)], axis=1)
        L, R = O.eig1d(U[0], U[1], b, g)
        np.testing.assert_allclose(L @ R, np.eye(2), atol=1e-13)
        u, c = U[1] / (U[0] - b), np.sqrt(g * (U[0] - b))
        np.testing.assert_allclose(L @ J @ R, np.diag([u - c, u + c]), atol=1e-12)


def test_flux_equals_conservative_form(oracle_mod):
    """The pre-balanced flux equals hu^2 + g h^2/2 minus the lake part g b^2/2 (eq. (2.2))."""
    O = oracle_mod
    g = 9.812
    for _ in range(5):
        b = RNG.uniform(-1, 1)
        h, u, v = RNG.uniform(0.5, 3), RNG.normal(), RNG.normal()
        F = O.flux2d(0, [h + b, h * u, h * v], b, g)
        np.testing.assert_allclose(F, [h * u, h * u * u + 0.5 * g * h * h - 0.5 * g * b * b, h * u * v], rtol=1e-12)
        F = O.flux2d(1, [h + b, h * u, h * v], b, g)
        np.testing.assert_allclose(F, [h * v, h * u * v, h * v * v + 0.5 * g * h * h - 0.5 * g * b * b], rtol=1e-12)


@pytest.mark.parametrize("lam,dt", [(-1.0, 0.3), (0.7, 0.1), (-3.0, 0.5)])
def test_ssprk3_linear(oracle_mod, lam, dt):
    """Eq. (2.11) on the scalar model R = lam * u: with the identity limiter one step is the
    third-order Taylor polynomial; with Lim(D) = mu D it follows the literal stage formulas."""
    O = oracle_mod
    z = lam * dt
    u, d = O.ssprk3_linear(lam, 1.0, dt, 1.3, -0.7)
    poly = 1 + z + z * z / 2 + z ** 3 / 6
    np.testing.assert_allclose([u, d], [1.3 * poly, -0.7 * poly], rtol=1e-14)
    mu = 0.8
    u, d = O.ssprk3_linear(lam, mu, dt, 1.0, 1.0)
    d1 = mu + z                      # D1 = D^{n,mod} + dt R_x(D^n)
    d2 = 0.75 * mu + 0.25 * (mu * d1 + z * d1)
    d3 = mu / 3 + 2.0 / 3 * (mu * d2 + z * d2)
    np.testing.assert_allclose(u, poly, rtol=1e-14)
    np.testing.assert_allclose(d, d3, rtol=1e-14)
    u, d = O.ssprk3_linear(lam, mu, dt, 1.0, 1.0, lim_first=True)
    d1 = mu * (1 + z)
    d2 = 0.75 * mu + 0.25 * mu * d1 * (1 + z)
    d3 = mu / 3 + 2.0 / 3 * mu * d2 * (1 + z)
    np.testing.assert_allclose(d, d3, rtol=1e-14)
