"""Pins of the oracle's forward-mode tangents (Dual numbers through the same scheme) and of its
single-precision entry points.

The tangents must be the derivatives of the oracle's own maps: central differences of the plain
FP64 functions converge to them at second order as the step shrinks (the nonlinear weights with
eps = 1e-6 make the maps' higher derivatives large, so the steps are small). At a lake at
rest the right-hand side vanishes for every bottom (the well-balance property of Sec. 2), so its
tangent along any bottom direction must vanish to round-off. The single-precision functions must
approximate the FP64 ones to float accuracy.
"""
import numpy as np
import pytest


def smooth_direction(I, pr, rng, fields=9):
    X, Y = I.nodes_2d(pr.nx, pr.ny, pr.domain)
    def bump():
        cx, cy = rng.uniform(0.4, 1.6, size=2)
        return np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * 0.15 ** 2))
    d = np.stack([rng.standard_normal() * bump() for _ in range(fields)])
    return d


def converges_to(jv, f):
    """Central differences (f(e) - f(-e)) / 2e for e = 1e-5, 1e-6, 1e-7 against the tangent jv:
    second-order decrease from 1e-5 to 1e-6, and agreement to 1e-6 at the best step."""
    errs = [rel((f(e) - f(-e)) / (2 * e), jv) for e in (1e-5, 1e-6, 1e-7)]
    assert errs[1] <= 0.05 * errs[0] or errs[0] <= 1e-9, errs
    assert min(errs) <= 1e-6, errs
    return errs


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def problem(O, I):
    pr = I.c5_adjoint(24)
    ax, ay = O.alpha(O.params_of(pr), pr.state, pr.b, pr.bx, pr.by)
    al = (1.1 * ax, 1.1 * ay)
    dt = 0.5 / (al[0] / pr.dx + al[1] / pr.dy)
    p = O.params_of(pr, flags=O.FIXED_DT | O.FIXED_ALPHA, fixed_dt=dt, alpha_x=(al[0],) * 3,
                    alpha_y=(al[1],) * 3)
    return pr, p, al


def test_rhs_jvp_is_the_derivative(oracle_mod, inputs_mod):
    O, I = oracle_mod, inputs_mod
    pr, p, al = problem(O, I)
    rng = np.random.default_rng(31)
    ds = smooth_direction(I, pr, rng)
    db, dbx, dby = smooth_direction(I, pr, rng, 3)
    _, jv = O.rhs_jvp(p, pr.state, ds, pr.b, pr.bx, pr.by, db, dbx, dby, al[0], al[1])
    # perturb state and bottom together through one packed vector
    n = pr.b.size
    x0 = np.concatenate([pr.state.ravel(), pr.b.ravel(), pr.bx.ravel(), pr.by.ravel()])
    dx = np.concatenate([ds.ravel(), db.ravel(), dbx.ravel(), dby.ravel()])

    def f(c):
        x = x0 + c * dx
        s = x[:9 * n].reshape(pr.state.shape)
        b, bx, by = (x[9 * n + k * n: 9 * n + (k + 1) * n].reshape(pr.b.shape) for k in range(3))
        return O.rhs(p, s, b, bx, by, al[0], al[1])
    converges_to(jv, f)


def test_limit_jvp_is_the_derivative(oracle_mod, inputs_mod):
    O, I = oracle_mod, inputs_mod
    pr, p, _ = problem(O, I)
    rng = np.random.default_rng(32)
    ds = smooth_direction(I, pr, rng)
    db = smooth_direction(I, pr, rng, 1)[0]
    z = np.zeros_like(pr.b)
    _, jv = O.limit_jvp(p, pr.state, ds, pr.b, pr.bx, pr.by, db, z, z)
    n = pr.b.size
    x0 = np.concatenate([pr.state.ravel(), pr.b.ravel()])
    dx = np.concatenate([ds.ravel(), db.ravel()])

    def f(c):
        x = x0 + c * dx
        return O.limit(p, x[:9 * n].reshape(pr.state.shape), x[9 * n:].reshape(pr.b.shape), pr.bx, pr.by)
    converges_to(jv, f)


def test_run_jvp_is_the_derivative(oracle_mod, inputs_mod):
    O, I = oracle_mod, inputs_mod
    pr, p, _ = problem(O, I)
    rng = np.random.default_rng(33)
    ds = smooth_direction(I, pr, rng)
    db, dbx, dby = smooth_direction(I, pr, rng, 3)
    _, jv = O.run_jvp(p, pr.state, ds, pr.b, pr.bx, pr.by, db, dbx, dby, 5)

    def f(c):
        return O.run(p, pr.state + c * ds, pr.b + c * db, pr.bx + c * dbx, pr.by + c * dby, nsteps=5)[0]
    converges_to(jv, f)


def test_rhs_tangent_along_the_bottom_vanishes_at_rest(oracle_mod, inputs_mod):
    O, I = oracle_mod, inputs_mod
    for pr in (I.c2_2d(32, "rest", ny=28), I.paper_lake_2d(24)):
        p = O.params_of(pr)
        rng = np.random.default_rng(34)
        db, dbx, dby = (rng.standard_normal(pr.b.shape) for _ in range(3))
        zs = np.zeros_like(pr.state)
        _, jb = O.rhs_jvp(p, pr.state, zs, pr.b, pr.bx, pr.by, db, dbx, dby, 3.5, 3.5)
        ds = rng.standard_normal(pr.state.shape)
        z = np.zeros_like(pr.b)
        _, js = O.rhs_jvp(p, pr.state, ds, pr.b, pr.bx, pr.by, z, z, z, 3.5, 3.5)
        assert np.abs(jb).max() <= 1e-11 * np.abs(js).max(), (pr.name, np.abs(jb).max(), np.abs(js).max())


def test_single_precision_functions(oracle_mod, inputs_mod):
    O, I = oracle_mod, inputs_mod
    pr = I.c2_2d(40, "smooth", ny=36)
    p = O.params_of(pr)
    r64 = O.rhs(p, pr.state, pr.b, pr.bx, pr.by)
    r32 = O.rhs_f32(p, pr.state, pr.b, pr.bx, pr.by)
    for g in ((0, 1, 2), (3, 4, 5)):  # U and U_x (the data vary in x only; U_y is round-off)
        g = list(g)
        assert rel(r32[g], r64[g]) <= 1e-3, rel(r32[g], r64[g])
    s64, t64, k64 = O.run(p, pr.state, pr.b, pr.bx, pr.by, nsteps=5)
    s32, t32, k32 = O.run_f32(p, pr.state, pr.b, pr.bx, pr.by, nsteps=5)
    assert k32 == k64 == 5 and abs(t32 - t64) <= 1e-6 * t64
    assert rel(s32, s64) <= 1e-4, rel(s32, s64)
    # the widened float run is the float delta of run_delta
    d32, _, _ = O.run_delta("f32", p, pr.state, pr.b, pr.bx, pr.by, nsteps=5)
    s0 = pr.state.astype(np.float32).astype(np.float64)
    assert np.abs((s32 - s0) - d32).max() <= 1e-6 * np.abs(d32).max()


@pytest.mark.slow
def test_c5_central_difference_epsilon_sweep(oracle_mod, inputs_mod):
    """On the adjoint workload (256^2, 100 steps at a fixed dt with frozen speeds, gauge misfit
    loss ~7e-11), the central difference of the loss along a smooth unit bottom direction
    approaches the oracle's forward-mode tangent at second order from large steps (truncation
    branch) and departs from it again below about 1e-4 (rounding branch: the loss's own rounding
    divided by the step). So a quotient at step 1e-6 is limited by the loss's rounding, not by the
    derivative it is compared with; at the best step the two agree to ~1e-10 (Sec. 4's workloads
    have no adjoint; the scheme differentiated is that of eq. (2.11) with readings R1, R22)."""
    O, I = oracle_mod, inputs_mod
    pr = I.c5_adjoint(256)
    nsteps = 100
    ax, ay = O.alpha(O.params_of(pr), pr.state, pr.b, pr.bx, pr.by)
    al = (1.1 * ax, 1.1 * ay)
    dt = 0.6 / (al[0] / pr.dx + al[1] / pr.dy)
    p = O.params_of(pr, flags=O.FIXED_DT | O.FIXED_ALPHA, fixed_dt=dt, alpha_x=(al[0],) * 3, alpha_y=(al[1],) * 3)
    g = pr.extra["gauges"]
    bt = pr.b + pr.extra["target_db"]
    tgt, _, _ = O.run(p, pr.state, bt, pr.bx + pr.extra["target_dbx"], pr.by + pr.extra["target_dby"], nsteps=nsteps)
    htgt = tgt[0][g[:, 0], g[:, 1]] - bt[g[:, 0], g[:, 1]]
    X, Y = I.nodes_2d(pr.nx, pr.ny, pr.domain)
    rng = np.random.default_rng(16)
    db, dbx, dby = np.zeros_like(X), np.zeros_like(X), np.zeros_like(X)
    for _ in range(4):  # a smooth direction with its analytic slopes
        cx, cy, w, a = rng.uniform(0.3, 1.7), rng.uniform(0.3, 1.7), rng.uniform(0.08, 0.2), rng.standard_normal()
        e = a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * w * w))
        db += e
        dbx += -e * (X - cx) / (w * w)
        dby += -e * (Y - cy) / (w * w)
    nrm = np.sqrt(np.sum(db ** 2))
    db, dbx, dby = db / nrm, dbx / nrm, dby / nrm

    def loss(c):
        s, _, _ = O.run(p, pr.state, pr.b + c * db, pr.bx + c * dbx, pr.by + c * dby, nsteps=nsteps)
        h = s[0][g[:, 0], g[:, 1]] - (pr.b + c * db)[g[:, 0], g[:, 1]]
        return float(np.sum((h - htgt) ** 2))

    sT, dT = O.run_jvp(p, pr.state, np.zeros_like(pr.state), pr.b, pr.bx, pr.by, db, dbx, dby, nsteps)
    h = sT[0][g[:, 0], g[:, 1]] - pr.b[g[:, 0], g[:, 1]]
    dh = dT[0][g[:, 0], g[:, 1]] - db[g[:, 0], g[:, 1]]
    tangent = float(np.sum(2.0 * (h - htgt) * dh))
    err = {}
    for e in (1e-2, 1e-4, 1e-6, 1e-8):
        err[e] = abs((loss(e) - loss(-e)) / (2 * e) - tangent) / abs(tangent)
    print("central difference vs tangent:", {f"{k:.0e}": f"{v:.2e}" for k, v in err.items()})
    assert err[1e-4] <= 1e-8                              # the derivative itself
    assert err[1e-2] >= 5 * err[1e-4]                     # truncation branch above
    assert err[1e-6] >= 10 * err[1e-4] and err[1e-8] >= 10 * err[1e-6]  # rounding branch below
