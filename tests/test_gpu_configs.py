"""The benchmark configurations end to end on the GPU against the oracle, at their stated sizes
(the 4096^2 dam break at a reduced grid): the 400^2 wall-bounded basin with the smooth
perturbation over 100 steps and with the strip over 200 steps, the dam break at 1024^2 over 50
steps, and 16 instances of the batched workload over 10 steps.

Error per equation group (U, V = U_x, Q = U_y): max |gpu - oracle| / max |oracle| over the
group. A group can be round-off itself: the y-derivatives of data perturbed along x only are
small, while each of their right-hand sides is a difference of fluxes and sources of size
g eta b_y / dy; two FP64 codes that round differently then agree only to that round-off,
accumulated over hundreds of stages. So, as for the one-step parity tests, each group must agree
to max(bar x group scale, 32 x the oracle's own round-off envelope): the spread of the oracle's
run when its initial state moves by about one unit in the last place. The whole state must
agree to the bar relative to its own scale. Bars: 1e-9 for the smooth perturbation after 100
steps, 1e-11 for the batch after 10 steps. The strip and the dam break carry discontinuities,
where the nonlinear weights respond to round-off differences between the two codes; their
errors are reported, with a loose bar that only catches a wrong scheme."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GROUPS = ((0, 1, 2), (3, 4, 5), (6, 7, 8))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def group_errs(a, b):
    return [np.abs(a[list(g)] - b[list(g)]).max() / max(np.abs(b[list(g)]).max(), 1e-300) for g in GROUPS]


def gpu_run(torch, pr, nsteps):
    from paper_2208_01260_amd.solver import Solver

    with Solver.from_problem(pr) as s:
        st = torch.from_numpy(pr.state).cuda().contiguous()
        t, k = s.run(st, nsteps=nsteps)
        return st.cpu().numpy(), t, k


def oracle_with_envelope(O, pr, nsteps, tag):
    """The oracle's run and the per-group spread of a second run from the initial state moved by
    about one unit in the last place (relative, seeded)."""
    p = O.params_of(pr)
    note(f"[{tag}] oracle on {O.get_threads()} threads")
    ref, t_ref, k_ref = O.run(p, pr.state, pr.b, pr.bx, pr.by, nsteps=nsteps)
    rng = np.random.default_rng(1)
    pert = pr.state * (1.0 + 2.0 ** -52 * rng.uniform(-1, 1, pr.state.shape))
    note(f"[{tag}] oracle envelope run")
    alt, _, _ = O.run(p, pert, pr.b, pr.bx, pr.by, nsteps=nsteps)
    env = [np.abs(alt[list(g)] - ref[list(g)]).max() for g in GROUPS]
    return ref, t_ref, k_ref, env


def judge(tag, got, ref, env, bar, loose=None):
    """Per group: err <= max(bar x scale, 32 x envelope) (or <= loose x scale when given); the
    whole state: err <= bar x scale (or loose)."""
    worst = 0.0
    lines = []
    for k, g in enumerate(GROUPS):
        g = list(g)
        scale = np.abs(ref[g]).max()
        err = np.abs(got[g] - ref[g]).max()
        allowed = loose * scale if loose else max(bar * scale, 32.0 * env[k])
        worst = max(worst, err / allowed)
        lines.append(f"{err / scale:.2e} (envelope {env[k] / scale:.2e})")
    whole = np.abs(got - ref).max() / np.abs(ref).max()
    note(f"[{tag}] group rel errors " + ", ".join(lines) + f"; whole state {whole:.2e}; err/allowed {worst:.3f}")
    return worst, whole


@pytest.mark.parametrize("variant,nsteps,bar,loose", [("smooth", 100, 1e-9, None), ("strip", 200, 1e-9, 1e-6)])
def test_c2_400_against_oracle(oracle_mod, inputs_mod, torch_cuda, variant, nsteps, bar, loose):
    pr = inputs_mod.c2_2d(400, variant)
    tag = f"c2 {variant}"
    note(f"[{tag}] 400x400, {nsteps} steps: GPU")
    got, t, k = gpu_run(torch_cuda, pr, nsteps)
    ref, t_ref, k_ref, env = oracle_with_envelope(oracle_mod, pr, nsteps, tag)
    worst, whole = judge(tag, got, ref, env, bar, loose)
    note(f"[{tag}] t {t!r} vs {t_ref!r}")
    assert k == k_ref == nsteps and abs(t - t_ref) <= 1e-12 * t_ref
    assert np.all(np.isfinite(got)) and worst <= 1 and whole <= (loose or bar)


def test_c3_dam_break_1024_50_steps(oracle_mod, inputs_mod, torch_cuda):
    pr = inputs_mod.c3_2d(1024)
    note("[c3] 1024x1024 dam break, 50 steps: GPU")
    got, t, k = gpu_run(torch_cuda, pr, 50)
    ref, t_ref, k_ref, env = oracle_with_envelope(oracle_mod, pr, 50, "c3")
    worst, whole = judge("c3", got, ref, env, 1e-9, 1e-6)
    note(f"[c3] t {t!r} vs {t_ref!r}")
    assert k == k_ref == 50 and abs(t - t_ref) <= 1e-12 * t_ref
    assert np.all(np.isfinite(got)) and worst <= 1 and whole <= 1e-6


def test_c4_sixteen_instances_against_oracle(oracle_mod, inputs_mod, torch_cuda):
    """The first 16 instances of the seeded 256-instance batch (sizes drawn from 64..512 per side),
    10 steps with per-instance CFL steps, each against the oracle run of that instance alone."""
    from paper_2208_01260_amd.solver import Batch

    probs = inputs_mod.c4_batch(256)[:16]
    note("[c4] 16 instances: " + " ".join(f"{p.nx}x{p.ny}" for p in probs))
    with Batch(probs) as bt:
        t_b = bt.run(10)
        got = [bt.states[i].cpu().numpy() for i in range(len(probs))]
    worst = 0.0
    for i, pr in enumerate(probs):
        ref, t_o, k, env = oracle_with_envelope(oracle_mod, pr, 10, f"c4 {i} {pr.nx}x{pr.ny}")
        w, whole = judge(f"c4 {i}", got[i], ref, env, 1e-11)
        worst = max(worst, w)
        assert k == 10 and abs(t_b[i] - t_o) <= 1e-13 * t_o
        assert w <= 1 and whole <= 1e-11, (i, w, whole)
    note(f"[c4] worst err/allowed {worst:.3f}")
