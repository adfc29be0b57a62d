"""GPU: the batched solver (swe_hweno_batch_*) through the C ABI.

Each instance of a batch must end bitwise equal to the plain solver run on that instance alone
with the same rows per wavefront march (the batch only changes which wavefront computes which
tile); with other rows the two differ by rounding only (the first y-interface of a march is a
separate copy of the same arithmetic, which the compiler may contract differently), and a batch
is also checked against the oracle directly. Instances are ragged: sizes that are not multiples
of the tile width or height, both boundary conditions, dx != dy.
"""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def ragged_instances(I):
    rng = np.random.default_rng(2208)
    out = [I.c4_instance(rng, sizes=(64, 93, 130, 161)) for _ in range(5)]
    out.append(I.c2_2d(77, "smooth", ny=41))        # periodic x, reflective y
    out.append(I.paper_accuracy_2d(61))             # periodic both
    out.append(I.c2_2d(4, "smooth"))                # smallest legal instance
    return out


def plain_run(torch, pr, nsteps, rows=16):
    """The plain solver on one instance; rows per march forced through SWE_HWENO_ROWS (None keeps
    the context's own choice)."""
    from paper_2208_01260_amd.solver import Solver

    old = os.environ.pop("SWE_HWENO_ROWS", None)
    try:
        if rows is not None:
            os.environ["SWE_HWENO_ROWS"] = str(rows)
        with Solver.from_problem(pr) as s:
            if rows is not None:
                assert s.tile()[1] == rows
            st = torch.from_numpy(pr.state).cuda().contiguous()
            t, k = s.run(st, nsteps=nsteps)
            assert k == nsteps
            return st.cpu().numpy(), t
    finally:
        os.environ.pop("SWE_HWENO_ROWS", None)
        if old is not None:
            os.environ["SWE_HWENO_ROWS"] = old


def group_err(a, b):
    worst = 0.0
    for g in ((0, 1, 2), (3, 4, 5), (6, 7, 8)):
        g = list(g)
        worst = max(worst, np.abs(a[g] - b[g]).max() / max(np.abs(b[g]).max(), 1e-300))
    return worst


@pytest.mark.parametrize("nsteps", [7, 20])
def test_batch_bitwise_equals_plain_solver(inputs_mod, torch_cuda, nsteps):
    from paper_2208_01260_amd.solver import Batch

    torch = torch_cuda
    probs = ragged_instances(inputs_mod)
    note(f"[batch] {len(probs)} instances, sizes {[(p.nx, p.ny) for p in probs]}, {nsteps} steps")
    with Batch(probs) as bt:
        t_b = bt.run(nsteps)
        got = [s.cpu().numpy() for s in bt.states]
    for i, pr in enumerate(probs):
        ref, t_p = plain_run(torch, pr, nsteps)
        assert np.array_equal(got[i], ref), (i, pr.name, np.abs(got[i] - ref).max())
        assert t_b[i] == t_p, (i, t_b[i], t_p)


def test_batch_rows_and_autotune_keep_results(inputs_mod, torch_cuda):
    from paper_2208_01260_amd.solver import Batch

    torch = torch_cuda
    probs = ragged_instances(inputs_mod)[:4]
    for rows in (1, 5, 64, 200):
        note(f"[batch] rows {rows}")
        with Batch(probs) as bt:
            bt.set_rows(rows)
            bt.run(5)
            for i, s in enumerate(bt.states):
                assert np.array_equal(s.cpu().numpy(), plain_run(torch, probs[i], 5, rows)[0]), (rows, i)
    Batch.tune_cache_clear()
    with Batch(probs) as bt:
        r = bt.autotune()
        note(f"[batch] autotune chose {r}")
        assert Batch.tune_cache_size() == 1
        assert r in (8, 12, 16, 24, 32, 48, 64)
        bt.run(5)
        for i, s in enumerate(bt.states):
            assert np.array_equal(s.cpu().numpy(), plain_run(torch, probs[i], 5, r)[0])
        # runs continue from the advanced states; a second run equals 10 plain steps
        bt.run(5)
        for i, pr in enumerate(probs):
            assert np.array_equal(bt.states[i].cpu().numpy(), plain_run(torch, pr, 10, r)[0]), i


def test_batch_autotune_cache(inputs_mod, torch_cuda):
    """A batch of a size class already tuned takes the cached rows; another class is tuned anew."""
    from paper_2208_01260_amd.solver import Batch

    torch = torch_cuda
    probs = ragged_instances(inputs_mod)[:4]
    Batch.tune_cache_clear()
    assert Batch.tune_cache_size() == 0
    with Batch(probs) as bt:
        r = bt.autotune()
    # the same instances in reverse order: same count, total nodes and extents
    with Batch(probs[::-1]) as bt:
        assert bt.autotune() == r
        assert Batch.tune_cache_size() == 1
        bt.run(3)
        for i, pr in enumerate(probs[::-1]):
            assert np.array_equal(bt.states[i].cpu().numpy(), plain_run(torch, pr, 3, r)[0]), i
    # one instance only: another class
    with Batch(probs[:1]) as bt:
        bt.autotune()
        assert Batch.tune_cache_size() == 2
    Batch.tune_cache_clear()
    assert Batch.tune_cache_size() == 0


def test_batch_rows_change_rounding_only(inputs_mod, torch_cuda):
    from paper_2208_01260_amd.solver import Batch

    torch = torch_cuda
    probs = ragged_instances(inputs_mod)
    with Batch(probs) as bt:
        bt.run(10)
        for i, pr in enumerate(probs):
            ref = plain_run(torch, pr, 10, rows=None)[0]
            got = bt.states[i].cpu().numpy()
            # relative to the whole state: a group that is round-off noise (the y-derivatives of
            # data that vary in x only) has no scale of its own
            err = np.abs(got - ref).max() / np.abs(ref).max()
            note(f"[batch] {pr.name} {pr.nx}x{pr.ny}: rows 16 vs own choice, state error {err:.2e}, "
                 f"group error {group_err(got, ref):.2e}")
            assert err <= 1e-11, (i, err)


def test_batch_against_oracle(oracle_mod, inputs_mod, torch_cuda):
    from paper_2208_01260_amd.solver import Batch

    O = oracle_mod
    rng = np.random.default_rng(7)
    probs = [inputs_mod.c4_instance(rng, sizes=(64, 96)) for _ in range(3)]
    with Batch(probs) as bt:
        t_b = bt.run(3)
        for i, pr in enumerate(probs):
            ref, t_o, k = O.run(O.params_of(pr), pr.state, pr.b, pr.bx, pr.by, nsteps=3)
            got = bt.states[i].cpu().numpy()
            assert k == 3 and abs(t_b[i] - t_o) <= 1e-14 * t_o
            for g in ((0, 1, 2), (3, 4, 5), (6, 7, 8)):
                g = list(g)
                err = np.abs(got[g] - ref[g]).max() / np.abs(ref[g]).max()
                assert err <= 1e-11, (i, g, err)


def test_batch_dry_instance_reported_others_advance(inputs_mod, torch_cuda):
    from paper_2208_01260_amd.solver import Batch, SweError

    torch = torch_cuda
    probs = ragged_instances(inputs_mod)[:3]
    bad = probs[1].state.copy()
    bad[0, 5, 7] = probs[1].b[5, 7] - 0.1
    states = [torch.from_numpy(p.state if i != 1 else bad).cuda().contiguous() for i, p in enumerate(probs)]
    with Batch(probs, states=states) as bt:
        with pytest.raises(SweError):
            bt.run(2)
        for i in (0, 2):
            assert np.array_equal(bt.states[i].cpu().numpy(), plain_run(torch, probs[i], 2)[0]), i
        # the dry node is met by the speeds of the initial state, before the first step: the
        # instance is stopped by that step's prologue and keeps its state unchanged
        assert np.array_equal(bt.states[1].cpu().numpy(), bad)
        bt.sync()  # the error was reported and cleared
