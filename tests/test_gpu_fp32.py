"""GPU: the single-precision variant (the _f32 entry points) through the C ABI.

FP32 results cannot match an FP64 oracle to FP64 tolerances; the bar is that the GPU's FP32
answer is about as accurate as the oracle's own FP32 answer (the same scheme run in float):
per equation group, max |gpu32 - oracle64| <= 4 max |oracle32 - oracle64| + 8 ulp(float) of the
group's scale. Lake at rest in FP32 must stay at the single-precision magnitudes the paper
prints (Tables 1-3, single-precision columns: within 5x).
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
F32_ULP = 2.0 ** -23


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def groups_of(pr):
    return ((0, 1, 2), (3, 4, 5), (6, 7, 8)) if pr.dim == 2 else ((0, 1), (2, 3))


def fp32_ratio(gpu, o32, o64, groups):
    """Worst over groups of |gpu - o64| / (4 |o32 - o64| + 8 ulp * scale) (<= 1 passes)."""
    worst = 0.0
    for g in groups:
        g = list(g)
        scale = np.abs(o64[g]).max()
        allowed = 4.0 * np.abs(o32[g] - o64[g]).max() + 8.0 * F32_ULP * scale
        worst = max(worst, np.abs(gpu[g] - o64[g]).max() / max(allowed, 1e-300))
    return worst


def solver32(pr):
    import torch

    from paper_2208_01260_amd.solver import Solver

    return Solver.from_problem(pr, dtype=torch.float32)


def to32(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda().contiguous()


def cases(I):
    return [
        ("c1_1d", I.c1_1d()),
        ("c2s_96x70", I.c2_2d(96, "smooth", ny=70)),
        ("c2strip_130x67", I.c2_2d(130, "strip", ny=67)),
        ("acc2d_periodic_61", I.paper_accuracy_2d(61)),
        ("c3_121x45", I.c3_2d(121, ny=45)),
        ("min_4x4_refl", I.c2_2d(4, "smooth")),
    ]


def test_fp32_rhs(oracle_mod, inputs_mod, torch_cuda):
    O, torch = oracle_mod, torch_cuda
    for name, pr in cases(inputs_mod):
        note(f"[fp32] rhs {name}")
        p = O.params_of(pr)
        o64 = O.rhs(p, pr.state, pr.b, pr.bx, pr.by)
        o32 = O.rhs_f32(p, pr.state, pr.b, pr.bx, pr.by)
        with solver32(pr) as s:
            got = s.rhs(to32(torch, pr.state)).double().cpu().numpy()
        r = fp32_ratio(got, o32, o64, groups_of(pr))
        note(f"[fp32] rhs {name}: ratio {r:.3f}")
        assert r <= 1.0, (name, r)


def test_fp32_steps(oracle_mod, inputs_mod, torch_cuda):
    O, torch = oracle_mod, torch_cuda
    for name, pr in cases(inputs_mod):
        for nsteps in (1, 20):
            p = O.params_of(pr)
            # inputs rounded to float on both sides
            s0 = np.asarray(pr.state, dtype=np.float32).astype(np.float64)
            o64, t64, _ = O.run(p, s0, pr.b, pr.bx, pr.by, nsteps=nsteps)
            o32, t32, _ = O.run_f32(p, s0, pr.b, pr.bx, pr.by, nsteps=nsteps)
            with solver32(pr) as s:
                st = to32(torch, s0)
                t, k = s.run(st, nsteps=nsteps)
                got = st.double().cpu().numpy()
            assert k == nsteps and abs(t - t64) <= 1e-5 * t64, (name, t, t64)
            r = fp32_ratio(got, o32, o64, groups_of(pr))
            note(f"[fp32] {name} {nsteps} steps: ratio {r:.3f}")
            assert r <= 1.0, (name, nsteps, r)


def lake_norms(torch, pr, t_end):
    with solver32(pr) as s:
        s0 = to32(torch, pr.state)
        st = s0.clone()
        t, _ = s.run(st, t_end=t_end)
        assert abs(t - t_end) <= 1e-6 * t_end
        d = (st.double() - s0.double()).cpu().numpy()
    return d


@pytest.mark.parametrize("kind,table", [("smooth", "table1_smooth_1d"), ("step", "table2_step_1d")])
def test_fp32_lake_at_rest_tables_1_2(inputs_mod, torch_cuda, kind, table):
    pr = inputs_mod.paper_lake_1d(kind)
    d = lake_norms(torch_cuda, pr, 0.5)
    for f, name in ((0, "h"), (1, "hu")):
        l1, li = np.mean(np.abs(d[f])), np.max(np.abs(d[f]))
        ref = GOLD[table]["f32"][name]
        note(f"[fp32] lake {kind} {name}: L1 {l1:.3g} Linf {li:.3g} (paper {ref[0]:.3g}, {ref[1]:.3g})")
        assert li > 0 and l1 <= 5 * ref[0] and li <= 5 * ref[1], (name, l1, li, ref)


def test_fp32_lake_at_rest_table_3(inputs_mod, torch_cuda):
    pr = inputs_mod.paper_lake_2d(200)
    d = lake_norms(torch_cuda, pr, 0.1)
    for f, name in ((0, "h"), (1, "hu"), (2, "hv")):
        l1, li = np.mean(np.abs(d[f])), np.max(np.abs(d[f]))
        ref = GOLD["table3_hump_2d"]["f32"][name]
        note(f"[fp32] lake 2D {name}: L1 {l1:.3g} Linf {li:.3g} (paper {ref[0]:.3g}, {ref[1]:.3g})")
        assert li > 0 and l1 <= 5 * ref[0] and li <= 5 * ref[1], (name, l1, li, ref)


def test_fp32_and_fp64_contexts_reject_each_others_calls(inputs_mod, torch_cuda):
    from paper_2208_01260_amd import _lib

    torch = torch_cuda
    pr = inputs_mod.c2_2d(32, "smooth")
    L = _lib.lib()
    with solver32(pr) as s32:
        st64 = torch.from_numpy(pr.state).cuda().contiguous()
        out64 = torch.empty_like(st64)
        assert L.swe_hweno_rhs(s32._ctx, st64.data_ptr(), out64.data_ptr(), -1.0, -1.0) == -1
        assert L.swe_hweno_run(s32._ctx, st64.data_ptr(), 1, 0.0, None, None) == -1
    from paper_2208_01260_amd.solver import Solver

    with Solver.from_problem(pr) as s64:
        st32 = to32(torch, pr.state)
        out32 = torch.empty_like(st32)
        assert L.swe_hweno_rhs_f32(s64._ctx, st32.data_ptr(), out32.data_ptr(), -1.0, -1.0) == -1
        assert L.swe_hweno_step_f32(s64._ctx, st32.data_ptr(), 0.0, None) == -1
