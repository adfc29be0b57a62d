"""Fifth-order convergence of the GPU solver itself (Sec. 4, the accuracy examples), measured the
way the oracle's own order pins measure it: self-convergence over x3 refinements, whose
cell-centred nodes nest, at a fixed dt proportional to dx^(5/3), so that the fifth-order spatial
error dominates the third-order time error. Full runs with the limiter, FP64."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _restrict(fine, k=3):
    """Nodes of a mesh refined k times (k odd) that coincide with the coarse nodes."""
    if fine.ndim == 2:
        return fine[:, k // 2::k]
    return fine[:, k // 2::k, k // 2::k]


def _run(torch, pr, T, c):
    from paper_2208_01260_amd.solver import FIXED_DT, Solver

    steps = int(np.ceil(T / (c * pr.dx ** (5.0 / 3.0))))
    with Solver.from_problem(pr, flags=FIXED_DT, fixed_dt=T / steps) as s:
        st = torch.from_numpy(pr.state).cuda().contiguous()
        t, k = s.run(st, nsteps=steps)
        assert abs(t - T) < 1e-12 and k == steps
        return st.cpu().numpy()


def _orders(S, fields):
    out = []
    for f in fields:
        a = S[0][f] - _restrict(S[1])[f]
        c = S[1][f] - _restrict(S[2])[f]
        out.append((np.log(np.mean(np.abs(a)) / np.mean(np.abs(c))) / np.log(3),
                    np.log(np.max(np.abs(a)) / np.max(np.abs(c))) / np.log(3)))
    return out


def test_fifth_order_2d(inputs_mod, torch_cuda):
    """Ex. 4.6 data (periodic), 45 -> 135 -> 405 nodes per side to t = 0.002: h, hu, hv (the
    oracle's pin on the same data measures L1 orders 4.86-5.33 and L-inf 4.58-5.30)."""
    S = [_run(torch_cuda, inputs_mod.paper_accuracy_2d(n), 0.002, 0.3) for n in (45, 135, 405)]
    orders = _orders(S, (0, 1, 2))
    print("2D orders (L1, L-inf) of h, hu, hv:", [(round(float(a), 2), round(float(b), 2)) for a, b in orders])
    for o1, oi in orders:
        assert o1 > 4.7 and oi > 4.4, orders


def test_fifth_order_1d(inputs_mod, torch_cuda):
    """Ex. 4.1 data (periodic), 45 -> 135 -> 405 nodes to t = 0.02: h and hu."""
    S = [_run(torch_cuda, inputs_mod.paper_accuracy_1d(n), 0.02, 0.5) for n in (45, 135, 405)]
    orders = _orders(S, (0, 1))
    print("1D orders (L1, L-inf) of h, hu:", [(round(float(a), 2), round(float(b), 2)) for a, b in orders])
    for o1, oi in orders:
        assert o1 > 4.4 and oi > 4.4, orders


@pytest.mark.parametrize("bc", [0, 1])
def test_mass_conserved_on_flat_bottom(inputs_mod, torch_cuda, bc):
    """With b = 0 the surface equation is a pure difference of interface fluxes, so the GPU run
    conserves sum(h) to round-off, across periodic wraps and reflective walls alike (2D: a
    moving 400 x 300 flat-bottom state, 50 steps at the CFL step; 1D: 1000 nodes, 200 steps)."""
    from dataclasses import replace

    from paper_2208_01260_amd.solver import Solver

    torch = torch_cuda
    I = inputs_mod
    pr = I.c2_2d(400, "flat", ny=300)
    pr = replace(pr, bc=(bc, bc))
    x = I.nodes_1d(1000, 0.0, 1.0)
    g = np.exp(-((x - 0.5) / 0.1) ** 2)
    st1 = np.stack([1.0 + 0.2 * g, 0.1 * np.sin(2 * np.pi * x), -0.2 * 2 * (x - 0.5) / 0.01 * g,
                    0.1 * 2 * np.pi * np.cos(2 * np.pi * x)])
    z = np.zeros(1000)
    pr1 = I.Problem("flat1d", 1, 1000, 1, (0.0, 1.0, 0.0, 1.0), (bc, 0), np.ascontiguousarray(st1), z, z, None)
    for p, nsteps in ((pr, 50), (pr1, 200)):
        assert not p.b.any()
        with Solver.from_problem(p) as s:
            st = torch.from_numpy(p.state).cuda().contiguous()
            s.run(st, nsteps=nsteps)
            out = st.cpu().numpy()
        m0, m1 = p.state[0].sum(), out[0].sum()
        moved = np.abs(out[0] - p.state[0]).max()
        print(f"dim {p.dim} bc {bc}: sum(h) {m0:.15e} -> {m1:.15e}, rel change {abs(m1 - m0) / m0:.1e}, "
              f"max |dh| {moved:.1e}")
        assert moved > 1e-4  # the state did evolve
        assert abs(m1 - m0) <= 1e-13 * m0
