"""Pins of the oracle's full scheme: well-balance (printed round-off magnitudes of Tables 1-3),
order of accuracy, symmetries, boundary conditions and conservation."""
import json
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
RNG = np.random.default_rng(2208)


def norms(d):
    return np.mean(np.abs(d)), np.max(np.abs(d))


# ------------------------------------------------------------------ well-balance (Sec. 2.1, 4.2, 4.7)
@pytest.mark.parametrize("kind,table", [("smooth", "table1_smooth_1d"), ("step", "table2_step_1d")])
def test_lake_at_rest_1d_matches_tables_1_2(oracle_mod, inputs_mod, kind, table):
    O, I = oracle_mod, inputs_mod
    pr = I.paper_lake_1d(kind)
    p = O.params_of(pr)
    for prec in ("f32", "f64", "f128"):
        d, t, k = O.run_delta(prec, p, pr.state, pr.b, pr.bx, t_end=0.5)
        assert abs(t - 0.5) < 1e-6 and k > 100
        for f, name in ((0, "h"), (1, "hu")):
            l1, li = norms(d[f])
            ref = GOLD[table][prec][name]
            assert li > 0, "round-off must be visible in this precision"
            if prec == "f32":
                # single precision: same or smaller magnitude than printed
                assert l1 <= 5 * ref[0] and li <= 5 * ref[1], (prec, name, l1, li, ref)
            else:
                assert ref[0] / 5 <= l1 <= 5 * ref[0], (prec, name, l1, ref)
                assert ref[1] / 5 <= li <= 5 * ref[1], (prec, name, li, ref)


@pytest.mark.slow
def test_lake_at_rest_2d_matches_table_3(oracle_mod, inputs_mod):
    O, I = oracle_mod, inputs_mod
    pr = I.paper_lake_2d(200)
    p = O.params_of(pr)
    d, t, k = O.run_delta("f64", p, pr.state, pr.b, pr.bx, pr.by, t_end=0.1)
    assert abs(t - 0.1) < 1e-12
    for f, name in ((0, "h"), (1, "hu"), (2, "hv")):
        l1, li = norms(d[f])
        ref = GOLD["table3_hump_2d"]["f64"][name]
        assert ref[0] / 5 <= l1 <= 5 * ref[0], (name, l1, ref)
        assert ref[1] / 5 <= li <= 5 * ref[1], (name, li, ref)
    # quadruple precision on a coarser mesh: the same 1e-33 magnitude
    pr = I.paper_lake_2d(40)
    d, t, k = O.run_delta("f128", O.params_of(pr), pr.state, pr.b, pr.bx, pr.by, t_end=0.1)
    for f, name in ((0, "h"), (1, "hu"), (2, "hv")):
        l1, li = norms(d[f])
        assert 0 < li <= 5 * GOLD["table3_hump_2d"]["f128"][name][1]


def random_lake(I, dim, n, bc, step_bottom=False):
    """Lake at rest (eta = const, m = w = 0, all derivatives of U zero) over a random bottom, drawn
    from a generator seeded by the case itself so that it does not depend on the test order."""
    rng = np.random.default_rng([2208, dim, n, bc, int(step_bottom)])
    if dim == 1:
        x = I.nodes_1d(n, 0.0, 1.0)
        b = 0.5 * np.sin(2 * np.pi * x + rng.uniform(0, 6)) + 0.3 * np.exp(-((x - 0.4) / 0.1) ** 2)
        bx = rng.normal(size=n)  # the balance holds for any B
        if step_bottom:
            b = np.where((x > 0.3) & (x < 0.6), 0.8, 0.0)
            bx = np.zeros(n)
        st = np.zeros((4, n))
        st[0] = 2.0 + rng.uniform(0, 1)
        return I.Problem("lake", 1, n, 1, (0.0, 1.0, 0.0, 1.0), (bc, 0), st, b, bx, None)
    X, Y = I.nodes_2d(n, n + 3, (0.0, 1.0, 0.0, 1.2))
    b = 0.6 * np.exp(-((X - 0.5) ** 2 + (Y - 0.6) ** 2) / 0.02) + 0.2 * np.sin(3 * X) * np.cos(2 * Y)
    if step_bottom:
        b = np.where(X + Y > 1.0, 0.7, 0.1)
    st = np.zeros((9,) + X.shape)
    st[0] = 1.5
    return I.Problem("lake", 2, n, n + 3, (0.0, 1.0, 0.0, 1.2), (bc, bc), st, b, rng.normal(size=X.shape),
                     rng.normal(size=X.shape))


@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("bc", [0, 1])
@pytest.mark.parametrize("step_bottom", [False, True])
def test_rhs_and_limiter_vanish_at_rest(oracle_mod, inputs_mod, dim, bc, step_bottom):
    """Propositions of Sec. 2.1 / 3: the residual of a lake at rest is round-off for any alpha,
    eps and bottom derivative; the limiter returns exactly zero derivatives (Sec. 2.2)."""
    O, I = oracle_mod, inputs_mod
    pr = random_lake(I, dim, 33, bc, step_bottom)
    for eps in (1e-6, 1e-10):
        p = O.params_of(pr, eps=eps)
        r = O.rhs(p, pr.state, pr.b, pr.bx, pr.by, 7.3, 5.1)
        # zero in exact arithmetic; the round-off bar is 256 units of 2^-53 of the flux magnitude
        # g eta (eta / 2 + |b| + |B|) / dx (the worst of 960 random lakes of this recipe is 132)
        e = pr.state[0].max()
        scale = 9.812 * e * (0.5 * e + np.abs(pr.b).max() + np.abs(pr.bx).max()) / min(pr.dx, pr.dy)
        assert np.abs(r).max() <= 256 * 2.0**-53 * scale, np.abs(r).max() / scale
        dm = O.limit(p, pr.state, pr.b, pr.bx, pr.by)
        assert np.all(dm == 0.0)


# ------------------------------------------------------------------ accuracy (Sec. 4.1, 4.6)
def _restrict(fine, k=3):
    """Nodes of a mesh refined k times (k odd) that coincide with the coarse nodes."""
    if fine.ndim == 2:
        return fine[:, k // 2::k]
    return fine[:, k // 2::k, k // 2::k]


def test_rhs_self_convergence_1d(oracle_mod, inputs_mod):
    O, I = oracle_mod, inputs_mod
    R = {}
    for n in (20, 60, 180):
        pr = I.paper_accuracy_1d(n)
        R[n] = O.rhs(O.params_of(pr), pr.state, pr.b, pr.bx, alpha_x=12.0)
    e1 = np.abs(R[20] - _restrict(R[60])).max(axis=1)
    e2 = np.abs(R[60] - _restrict(R[180])).max(axis=1)
    order = np.log(e1 / e2) / np.log(3)
    assert np.all(order[:2] > 4.7), order  # U equations: fifth order (sixth for the linear part)
    assert np.all(order[2:] > 4.5), order  # V equations: Q' of the quintic, fifth order


def test_rhs_self_convergence_2d(oracle_mod, inputs_mod):
    O, I = oracle_mod, inputs_mod
    R = {}
    for n in (20, 60, 180):
        pr = I.paper_accuracy_2d(n)
        R[n] = O.rhs(O.params_of(pr), pr.state, pr.b, pr.bx, pr.by, 25.0, 25.0)
    e1 = np.abs(R[20] - _restrict(R[60])).max(axis=(1, 2))
    e2 = np.abs(R[60] - _restrict(R[180])).max(axis=(1, 2))
    order = np.log(e1 / e2) / np.log(3)
    assert np.all(order[:3] > 4.8), order
    assert np.all(order[3:] > 3.7), order  # the mixed four-point terms are fourth order


def test_limiter_perturbation_is_fourth_order(oracle_mod, inputs_mod):
    """|V^mod - V| = O(dx^4) on smooth data (Sec. 2.2)."""
    O, I = oracle_mod, inputs_mod
    err = []
    for n in (40, 120):
        pr = I.paper_accuracy_1d(n)
        dm = O.limit(O.params_of(pr), pr.state, pr.b, pr.bx)
        err.append(np.abs(dm - pr.state[2:]).max())
    assert np.log(err[0] / err[1]) / np.log(3) > 3.7, err


@pytest.mark.slow
@pytest.mark.parametrize("eps,min_order", [(1e-6, 4.4), (1e30, 4.85)])
def test_full_run_fifth_order_1d(oracle_mod, inputs_mod, eps, min_order):
    """Ex. 4.1 data: self-convergence of h and hu at fifth order (dt ~ dx^(5/3), x3 refinement so
    that cell-centred nodes nest). The run stops at t = 0.02: by t = 0.1 the hu gradient has grown
    fifteen-fold and meshes below ~10^3 nodes are not yet asymptotic. eps = 1e30 gives the linear
    weights (3/10, 3/10, 4/10), i.e. the underlying quintic Hermite scheme."""
    O, I = oracle_mod, inputs_mod
    S, T = {}, 0.02
    for n in (45, 135, 405):
        pr = I.paper_accuracy_1d(n)
        steps = int(np.ceil(T / (0.5 * pr.dx ** (5.0 / 3.0))))
        p = O.params_of(pr, flags=O.FIXED_DT, fixed_dt=T / steps, eps=eps)
        S[n], t, k = O.run(p, pr.state, pr.b, pr.bx, nsteps=steps)
        assert abs(t - T) < 1e-12 and k == steps
    for f in (0, 1):  # eta - b = h (b is fixed) and hu
        a = S[45][f] - _restrict(S[135])[f]
        c = S[135][f] - _restrict(S[405])[f]
        for norm in (lambda v: np.mean(np.abs(v)), lambda v: np.max(np.abs(v))):
            assert np.log(norm(a) / norm(c)) / np.log(3) > min_order


# ------------------------------------------------------------------ symmetries and boundaries
def _smooth2d(I, nx, ny, bc=(0, 0)):
    pr = I.paper_accuracy_2d(nx) if nx == ny else None
    if pr is None or bc != (0, 0):
        X, Y = I.nodes_2d(nx, ny, (0.0, 1.0, 0.0, 1.0))
        f = lambda x, y: 2.0 + 0.3 * np.sin(2 * np.pi * x + 0.4) * np.cos(2 * np.pi * y)
        st = np.stack([f(X, Y), 0.2 * np.sin(2 * np.pi * Y), 0.1 * np.cos(2 * np.pi * X)] +
                      [RNG.normal(size=X.shape) for _ in range(6)])
        b = 0.3 * np.cos(2 * np.pi * X) * np.sin(2 * np.pi * Y + 1)
        pr = I.Problem("s", 2, nx, ny, (0.0, 1.0, 0.0, 1.0), bc, st, b, RNG.normal(size=X.shape),
                       RNG.normal(size=X.shape))
    return pr


def test_transpose_symmetry_2d(oracle_mod, inputs_mod):
    """x <-> y: (m, w) swap, V <-> Q with components permuted, b_x <-> b_y; the y-sweep is the
    transpose of the x-sweep."""
    O, I = oracle_mod, inputs_mod
    pr = _smooth2d(I, 24, 24, bc=(1, 1))
    p = O.params_of(pr)
    r = O.rhs(p, pr.state, pr.b, pr.bx, pr.by, 4.0, 6.0)
    perm = [0, 2, 1, 6, 8, 7, 3, 5, 4]
    st = np.ascontiguousarray(pr.state[perm].transpose(0, 2, 1))
    rt = O.rhs(p, st, pr.b.T.copy(), pr.by.T.copy(), pr.bx.T.copy(), 6.0, 4.0)
    np.testing.assert_allclose(rt, r[perm].transpose(0, 2, 1), rtol=0, atol=1e-13 * np.abs(r).max())


@pytest.mark.parametrize("dim", [1, 2])
def test_mirror_symmetry(oracle_mod, inputs_mod, dim):
    """x -> -x maps the "+" reconstruction onto the "-" one (Sec. 2.1, mirror symmetric)."""
    O, I = oracle_mod, inputs_mod
    if dim == 1:
        pr = I.c1_1d(64)
        par = np.array([1, -1, -1, 1])[:, None]
        st = np.ascontiguousarray(pr.state[:, ::-1] * par)
        p = O.params_of(pr)
        r = O.rhs(p, pr.state, pr.b, pr.bx, alpha_x=5.0)
        rm = O.rhs(p, st, pr.b[::-1].copy(), -pr.bx[::-1].copy(), alpha_x=5.0)
        np.testing.assert_allclose(rm, r[:, ::-1] * par, rtol=0, atol=1e-12 * np.abs(r).max())
        return
    pr = _smooth2d(I, 20, 26, bc=(1, 0))
    par = np.array([1, -1, 1, -1, 1, -1, 1, -1, 1])[:, None, None]
    st = np.ascontiguousarray(pr.state[:, :, ::-1] * par)
    p = O.params_of(pr)
    r = O.rhs(p, pr.state, pr.b, pr.bx, pr.by, 5.0, 5.0)
    rm = O.rhs(p, st, pr.b[:, ::-1].copy(), -pr.bx[:, ::-1].copy(), pr.by[:, ::-1].copy(), 5.0, 5.0)
    np.testing.assert_allclose(rm, r[:, :, ::-1] * par, rtol=0, atol=1e-12 * np.abs(r).max())


def test_1d_embedding_in_2d(oracle_mod, inputs_mod):
    """y-independent 2D data with w = 0, Q = 0, b_y = 0 evolve exactly as the 1D scheme."""
    O, I = oracle_mod, inputs_mod
    pr1 = I.c1_1d(48)
    ny = 6
    st = np.zeros((9, ny, 48))
    st[0], st[1], st[3], st[4] = pr1.state[0], pr1.state[1], pr1.state[2], pr1.state[3]
    b = np.tile(pr1.b, (ny, 1))
    bx = np.tile(pr1.bx, (ny, 1))
    p2 = O.make_params(2, 48, ny, (0.0, 1.0, 0.0, 0.5))
    p1 = O.params_of(pr1)
    r1 = O.rhs(p1, pr1.state, pr1.b, pr1.bx, alpha_x=3.5)
    r2 = O.rhs(p2, st, b, bx, np.zeros_like(b), 3.5, 1.0)
    for j in range(ny):
        np.testing.assert_allclose(r2[[0, 1, 3, 4], j], r1, rtol=0, atol=1e-14 * np.abs(r1).max())
    assert np.all(r2[[2, 5, 6, 7, 8]] == 0)
    s1, dt1 = O.step(O.params_of(pr1, flags=O.FIXED_DT, fixed_dt=1e-3), pr1.state, pr1.b, pr1.bx, dt=1e-3)
    s2, _ = O.step(O.make_params(2, 48, ny, (0.0, 1.0, 0.0, 0.5), flags=O.FIXED_DT, fixed_dt=1e-3), st, b, bx,
                   np.zeros_like(b), dt=1e-3)
    np.testing.assert_allclose(s2[[0, 1, 3, 4], 2], s1, rtol=0, atol=1e-14 * np.abs(s1).max())


@pytest.mark.parametrize("dim", [1, 2])
def test_reflective_equals_periodic_even_extension(oracle_mod, inputs_mod, dim):
    """A reflective wall is the mirror plane of a doubled periodic domain: the parity of every
    field across the wall (eta, w, b even; m, eta_x, w_x, b_x odd across x) is what the
    reflective ghost nodes apply."""
    O, I = oracle_mod, inputs_mod
    if dim == 1:
        n = 40
        x = I.nodes_1d(n, 0.0, 1.0)
        st = np.stack([2.0 + 0.1 * np.cos(3 * x), 0.3 * np.sin(2 * x) + 0.1, RNG.normal(size=n), RNG.normal(size=n)])
        b, bx = 0.2 * np.cos(5 * x), RNG.normal(size=n)
        par = np.array([1, -1, -1, 1])[:, None]
        ext = np.concatenate([st, (st * par)[:, ::-1]], axis=1)
        bext, bxext = np.concatenate([b, b[::-1]]), np.concatenate([bx, -bx[::-1]])
        pr = O.make_params(1, n, 1, (0.0, 1.0, 0, 1), bc=(1, 0))
        pp = O.make_params(1, 2 * n, 1, (0.0, 2.0, 0, 1), bc=(0, 0))
        r = O.rhs(pr, st, b, bx, alpha_x=5.0)
        re = O.rhs(pp, ext, bext, bxext, alpha_x=5.0)
        np.testing.assert_allclose(re[:, :n], r, rtol=0, atol=1e-12 * np.abs(r).max())
        s, _ = O.step(pr, st, b, bx)
        se, _ = O.step(pp, ext, bext, bxext)
        np.testing.assert_allclose(se[:, :n], s, rtol=0, atol=1e-12 * np.abs(s).max())
        return
    n, m = 16, 18
    X, Y = I.nodes_2d(n, m, (0.0, 1.0, 0.0, 1.0))
    st = np.stack([2.0 + 0.1 * np.cos(3 * X + Y), 0.3 * np.sin(2 * X) + 0.1 * Y, 0.2 * np.cos(Y) * X] +
                  [RNG.normal(size=X.shape) for _ in range(6)])
    b, bx, by = 0.2 * np.cos(5 * X) * np.sin(2 * Y), RNG.normal(size=X.shape), RNG.normal(size=X.shape)
    px = np.array([1, -1, 1, -1, 1, -1, 1, -1, 1])[:, None, None]
    py = np.array([1, 1, -1, 1, 1, -1, -1, -1, 1])[:, None, None]
    ex = np.concatenate([st, (st * px)[:, :, ::-1]], axis=2)
    ext = np.concatenate([ex, (ex * py)[:, ::-1, :]], axis=1)

    def ext2(f, sx, sy):
        e = np.concatenate([f, sx * f[:, ::-1]], axis=1)
        return np.concatenate([e, sy * e[::-1, :]], axis=0)

    pr = O.make_params(2, n, m, (0.0, 1.0, 0.0, 1.0), bc=(1, 1))
    pp = O.make_params(2, 2 * n, 2 * m, (0.0, 2.0, 0.0, 2.0), bc=(0, 0))
    r = O.rhs(pr, st, b, bx, by, 5.0, 4.0)
    re = O.rhs(pp, np.ascontiguousarray(ext), ext2(b, 1, 1), ext2(bx, -1, 1), ext2(by, 1, -1), 5.0, 4.0)
    np.testing.assert_allclose(re[:, :m, :n], r, rtol=0, atol=1e-12 * np.abs(r).max())
    dm = O.limit(pr, st, b, bx, by)
    dme = O.limit(pp, np.ascontiguousarray(ext), ext2(b, 1, 1), ext2(bx, -1, 1), ext2(by, 1, -1))
    np.testing.assert_allclose(dme[:, :m, :n], dm, rtol=0, atol=1e-12 * np.abs(dm).max())


@pytest.mark.parametrize("dim,bc", [(1, 0), (1, 1), (2, 0), (2, 1)])
def test_mass_conserved_on_flat_bottom(oracle_mod, inputs_mod, dim, bc):
    """With b = 0 the eta-equation is a pure flux difference: sum(h) is conserved to round-off."""
    O, I = oracle_mod, inputs_mod
    if dim == 1:
        n = 64
        x = I.nodes_1d(n, 0.0, 1.0)
        st = np.stack([1.0 + 0.2 * np.exp(-((x - 0.5) / 0.1) ** 2), 0.1 * np.sin(2 * np.pi * x),
                       np.zeros(n), np.zeros(n)])
        st[2] = -0.2 * 2 * (x - 0.5) / 0.01 * np.exp(-((x - 0.5) / 0.1) ** 2)
        st[3] = 0.1 * 2 * np.pi * np.cos(2 * np.pi * x)
        p = O.make_params(1, n, 1, (0.0, 1.0, 0, 1), bc=(bc, 0))
        b = np.zeros(n)
        s, t, k = O.run(p, st, b, b, nsteps=20)
        assert abs(s[0].sum() - st[0].sum()) <= 1e-13 * st[0].sum()
        return
    pr = I.c2_2d(40, "flat")
    p = O.params_of(pr, bc=(bc, bc))
    s, t, k = O.run(p, pr.state, pr.b, pr.bx, pr.by, nsteps=10)
    assert abs(s[0].sum() - pr.state[0].sum()) <= 1e-13 * pr.state[0].sum()


def test_flop_count_is_stable(oracle_mod, inputs_mod):
    """The counted arithmetic of one 2D right-hand side, per node (used for the roofline)."""
    O, I = oracle_mod, inputs_mod
    per = []
    for n in (64, 128):
        pr = I.c2_2d(n, "smooth")
        c = O.count_rhs(O.params_of(pr), pr.state, pr.b, pr.bx, pr.by, 3.0, 3.0)
        per.append((c["add"] + c["mul"] + c["div"] + c["sqrt"]) / n ** 2)
    assert 1500 < per[1] < 4000
    assert abs(per[0] - per[1]) / per[1] < 0.05


def test_stored_flop_counts_are_current(oracle_mod):
    """tests/golden/flop_counts.json (read by the benchmark's roofline) matches the oracle."""
    import importlib.util
    here = os.path.join(os.path.dirname(__file__), "golden")
    spec = importlib.util.spec_from_file_location("mk", os.path.join(here, "make_flop_counts.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    stored = json.load(open(os.path.join(here, "flop_counts.json")))
    fresh = mk.counts()
    # (a one-time handful of constant initialisations may land in either count)
    assert abs(stored["rhs_flops_per_node"] - fresh["rhs_flops_per_node"]) < 0.01
    assert abs(stored["limiter_flops_per_node"] - fresh["limiter_flops_per_node"]) < 0.01


# ------------------------------------------------------------------ the 2D limiter in y, alpha and dt
def _rough2d(nx, ny, domain, bc, seed):
    """Non-smooth 2D data (a jump in the surface along a slanted line, random momenta of both
    signs, random derivatives), so that the limiter's nonlinear weights are far from linear and
    depend on the characteristic decomposition."""
    rng = np.random.default_rng(seed)
    x = domain[0] + (np.arange(nx) + 0.5) * (domain[1] - domain[0]) / nx
    y = domain[2] + (np.arange(ny) + 0.5) * (domain[3] - domain[2]) / ny
    X, Y = np.meshgrid(x, y, indexing="xy")
    b = 0.3 * np.exp(-((X - 0.4) ** 2 + (Y - 0.7) ** 2) / 0.05)
    eta = np.where(X + 0.6 * Y > 0.8, 2.0, 1.4) + 0.05 * rng.normal(size=X.shape)
    st = np.stack([eta, 0.4 * rng.normal(size=X.shape), 0.4 * rng.normal(size=X.shape)] +
                  [rng.normal(size=X.shape) for _ in range(6)])
    return st, b, rng.normal(size=X.shape), rng.normal(size=X.shape)


@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (1, 0)])
def test_limiter_transpose_symmetry_2d(oracle_mod, bc):
    """x <-> y for the limiter (Sec. 2.2, applied dimension by dimension in Sec. 3): Q^mod of a
    state is V^mod of the transposed state, with the y-eigenvectors of the node playing the
    x-eigenvectors' part. Unequal grids and spacings catch a dx/dy or nx/ny mix-up."""
    O = oracle_mod
    nx, ny, dom = 23, 17, (0.0, 1.0, 0.0, 1.3)
    st, b, bx, by = _rough2d(nx, ny, dom, bc, [2208, 7, bc[0], bc[1]])
    p = O.make_params(2, nx, ny, dom, bc=bc)
    dm = O.limit(p, st, b, bx, by)
    assert np.abs(dm - st[3:]).max() > 1e-3  # the limiter acts on this data
    perm = [0, 2, 1, 6, 8, 7, 3, 5, 4]
    stT = np.ascontiguousarray(st[perm].transpose(0, 2, 1))
    pT = O.make_params(2, ny, nx, (dom[2], dom[3], dom[0], dom[1]), bc=(bc[1], bc[0]))
    dmT = O.limit(pT, stT, b.T.copy(), by.T.copy(), bx.T.copy())
    dperm = [3, 5, 4, 0, 2, 1]
    np.testing.assert_allclose(dmT, dm[dperm].transpose(0, 2, 1), rtol=0, atol=1e-13 * np.abs(dm).max())


@pytest.mark.parametrize("bc", [0, 1])
def test_1d_embedding_in_2d_along_y(oracle_mod, inputs_mod, bc):
    """x-independent 2D data with m = 0, V = 0 and b_x = 0 evolve along y exactly as the 1D scheme
    does along x (Sec. 2 against Sec. 3): (eta, w, H2, W2, b, b_y) play (eta, m, H, M, b, B). This
    pins the y-sweep, the y-limiter (y-eigenvectors, y-neighbours, dy) and the y-walls against the
    1D scheme, which the tables and the convergence tests pin. A jump makes the limiter act."""
    O, I = oracle_mod, inputs_mod
    ny, nx = 48, 5
    y = I.nodes_1d(ny, 0.0, 1.3)
    rng = np.random.default_rng([2208, 11, bc])
    b1 = 0.2 * np.cos(2 * np.pi * y / 1.3) + 0.1 * np.sin(4 * np.pi * y / 1.3 + 0.3)
    B1 = rng.normal(size=ny)
    st1 = np.stack([np.where((y > 0.4) & (y < 0.8), 2.0, 1.5) + 0.02 * rng.normal(size=ny),
                    0.3 * rng.normal(size=ny), rng.normal(size=ny), rng.normal(size=ny)])
    p1 = O.make_params(1, ny, 1, (0.0, 1.3, 0.0, 1.0), bc=(bc, 0))
    st = np.zeros((9, ny, nx))
    st[0], st[2], st[6], st[8] = (np.repeat(st1[k][:, None], nx, axis=1) for k in range(4))
    b = np.repeat(b1[:, None], nx, axis=1)
    by = np.repeat(B1[:, None], nx, axis=1)
    p2 = O.make_params(2, nx, ny, (0.0, 0.7, 0.0, 1.3), bc=(0, bc))
    r1 = O.rhs(p1, st1, b1, B1, alpha_x=3.5)
    r2 = O.rhs(p2, st, b, np.zeros_like(b), by, 1.0, 3.5)
    d1 = O.limit(p1, st1, b1, B1)
    d2 = O.limit(p2, st, b, np.zeros_like(b), by)
    assert np.abs(d1 - st1[2:]).max() > 1e-3  # the limiter acts on this data
    for i in range(nx):
        np.testing.assert_allclose(r2[[0, 2, 6, 8], :, i], r1, rtol=0, atol=1e-14 * np.abs(r1).max())
        np.testing.assert_allclose(d2[[3, 5], :, i], d1, rtol=0, atol=1e-14 * np.abs(d1).max())
    assert np.all(r2[[1, 3, 4, 5, 7]] == 0) and np.all(d2[[0, 1, 2, 4]] == 0)
    s1, _ = O.step(O.make_params(1, ny, 1, (0.0, 1.3, 0.0, 1.0), bc=(bc, 0), flags=O.FIXED_DT, fixed_dt=2e-3),
                   st1, b1, B1, dt=2e-3)
    s2, _ = O.step(O.make_params(2, nx, ny, (0.0, 0.7, 0.0, 1.3), bc=(0, bc), flags=O.FIXED_DT, fixed_dt=2e-3),
                   st, b, np.zeros_like(b), by, dt=2e-3)
    for i in range(nx):
        np.testing.assert_allclose(s2[[0, 2, 6, 8], :, i], s1, rtol=0, atol=1e-14 * np.abs(s1).max())


def test_limiter_perturbation_is_fourth_order_2d(oracle_mod, inputs_mod):
    """|V^mod - V| and |Q^mod - Q| = O(dx^4) on the smooth data of Ex. 4.6 (Sec. 2.2 and 3),
    separately for the x- and the y-limited derivatives."""
    O, I = oracle_mod, inputs_mod
    ev, eq = [], []
    for n in (90, 270):  # (30 -> 90 is pre-asymptotic for the x-derivatives: order 3.2)
        pr = I.paper_accuracy_2d(n)
        dm = O.limit(O.params_of(pr), pr.state, pr.b, pr.bx, pr.by)
        ev.append(np.abs(dm[:3] - pr.state[3:6]).max())
        eq.append(np.abs(dm[3:] - pr.state[6:9]).max())
    assert np.log(ev[0] / ev[1]) / np.log(3) > 3.7, ev
    assert np.log(eq[0] / eq[1]) / np.log(3) > 3.7, eq


@pytest.mark.slow
def test_full_run_fifth_order_2d(oracle_mod, inputs_mod):
    """Ex. 4.6 data: self-convergence of h, hu, hv over a full run with the limiter at fifth order
    (Sec. 4, second accuracy example). dt ~ dx^(5/3) and x3 refinement (cell-centred nodes nest).
    15 -> 45 -> 135 is pre-asymptotic for this data (L-inf orders 2.8-3.8); 45 -> 135 -> 405 gives
    L1 orders 4.86-5.33 and L-inf 4.58-5.30."""
    O, I = oracle_mod, inputs_mod
    S, T = {}, 0.002
    for n in (45, 135, 405):
        pr = I.paper_accuracy_2d(n)
        steps = int(np.ceil(T / (0.3 * pr.dx ** (5.0 / 3.0))))
        p = O.params_of(pr, flags=O.FIXED_DT, fixed_dt=T / steps)
        S[n], t, k = O.run(p, pr.state, pr.b, pr.bx, pr.by, nsteps=steps)
        assert abs(t - T) < 1e-12 and k == steps
    for f in (0, 1, 2):  # eta - b = h (b is fixed), hu, hv
        a = S[45][f] - _restrict(S[135])[f]
        c = S[135][f] - _restrict(S[405])[f]
        o1 = np.log(np.mean(np.abs(a)) / np.mean(np.abs(c))) / np.log(3)
        oi = np.log(np.max(np.abs(a)) / np.max(np.abs(c))) / np.log(3)
        assert o1 > 4.7 and oi > 4.4, (f, o1, oi)


def test_alpha_and_dt_golden(oracle_mod):
    """Hand-computed Lax-Friedrichs speeds and CFL step of two-state data (readings R1 and R11,
    tests/golden/alpha_dt_two_state.json): the x- and y-maxima are attained at different nodes,
    so a per-node sum, a wrong sound speed or a swapped spacing gives another step. The
    right-hand side without given speeds equals the one with the golden speeds."""
    O = oracle_mod
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "alpha_dt_two_state.json")))
    for case in gold["cases"]:
        nx, ny, dom = case["nx"], case["ny"], tuple(case["domain"])
        dim = case["dim"]
        p = O.make_params(dim, nx, ny, dom, g=case["g"], cfl=case["cfl"])
        shape = (nx,) if dim == 1 else (ny, nx)
        left = (np.arange(nx) < case["split"]) if dim == 1 else (np.arange(nx)[None, :] < case["split"]) & np.ones(shape, bool)
        A, B = case["left"], case["right"]
        nf = 4 if dim == 1 else 9
        st = np.zeros((nf,) + shape)
        st[0] = np.where(left, A["eta"], B["eta"])
        st[1] = np.where(left, A["m"], B["m"])
        if dim == 2:
            st[2] = np.where(left, A["w"], B["w"])
        b = np.full(shape, case["b"])
        z = np.zeros(shape)
        by = z if dim == 2 else None
        ax, ay = O.alpha(p, st, b, z, by)
        assert ax == pytest.approx(case["alpha_x"], rel=1e-15, abs=0)
        if dim == 2:
            assert ay == pytest.approx(case["alpha_y"], rel=1e-15, abs=0)
        _, dt = O.step(p, st, b, z, by)
        assert dt == pytest.approx(case["dt"], rel=2e-16, abs=0)
        r = O.rhs(p, st, b, z, by)
        rg = O.rhs(p, st, b, z, by, case["alpha_x"], case.get("alpha_y", 1.0))
        np.testing.assert_array_equal(r, rg)
        # the last step of a run is clipped to the final time
        t_end = 0.4 * case["dt"]
        _, t, k = O.run(p, st, b, z, by, t_end=t_end)
        assert k == 1 and t == t_end
