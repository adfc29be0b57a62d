"""Boundary behaviour of the C ABI on the GPU: the arithmetic building blocks against IEEE
division and square root, refusal of a NaN Lax-Friedrichs speed, and the bare right-hand side's
report of dry or non-finite input (through swe_hweno_sync, or at once with SWE_CHECK_DRY)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _logspace_normals(rng, n, lo, hi, signed=False):
    """Random doubles with log2|x| uniform in [lo, hi] and random mantissas."""
    x = np.ldexp(rng.uniform(1.0, 2.0, n), rng.integers(lo, hi, n))
    if signed:
        x *= rng.choice([-1.0, 1.0], n)
    return x


def test_math_building_blocks_match_ieee(torch_cuda):
    """rcp (two Newton steps on the hardware estimate), sqrt_pos (Goldschmidt step and two
    corrections) and div3 (product and one FMA correction) give the correctly rounded IEEE
    result on random arguments across their stated domains, tiny and huge normals included:
    1/x for 2^-1021 <= |x| <= 2^1021, sqrt(x) for 2^-1000 <= x <= the largest double, x/3 for
    2^-1000 <= |x| <= the largest double and x = 0 (as +0 for -0). (Below 2^-1000 the corrections' residuals
    fall among the subnormals and the last bit can differ; the solver's depths, speeds and
    states are nowhere near there.)"""
    from paper_2208_01260_amd import _lib

    torch = torch_cuda
    L = _lib.lib()
    rng = np.random.default_rng(2208)
    n = 1 << 22
    big = np.finfo(np.float64).max
    cases = {
        0: (np.concatenate([_logspace_normals(rng, n, -1021, 1021, True),
                            np.array([1.0, -1.0, 3.0, 2.0 ** -1021, 2.0 ** 1021, np.nextafter(2.0, 0)])]),
            lambda x: 1.0 / x),
        1: (np.concatenate([_logspace_normals(rng, n, -1000, 1023),
                            np.array([1.0, 2.0, 4.0, 2.0 ** -1000, big, 9.812 * 10.0])]),
            np.sqrt),
        2: (np.concatenate([_logspace_normals(rng, n, -1000, 1023, True),
                            np.array([0.0, -0.0, 3.0, 1.0, -1.0, 2.0 ** -1000, big, -big])]),
            lambda x: x / 3.0),
    }
    bad_all = {}
    for which, (x, ref) in cases.items():
        xd = torch.from_numpy(x).cuda()
        yd = torch.empty_like(xd)
        rc = L.swe_hweno_math_check(which, xd.data_ptr(), yd.data_ptr(), x.size,
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0, _lib.strerror(rc)
        y = yd.cpu().numpy()
        want = ref(x)
        bad = np.flatnonzero(y != want)  # numerical equality (div3 returns +0 for -0)
        print(f"building block {which}: {x.size} arguments, {bad.size} differ from IEEE"
              + (f" (smallest such |x| {np.abs(x[bad]).min():.3e})" if bad.size else ""), flush=True)
        if bad.size:
            bad_all[which] = (x[bad[:5]], y[bad[:5]], want[bad[:5]])
    assert not bad_all, bad_all


def test_rhs_refuses_nan_speed(torch_cuda, inputs_mod):
    from paper_2208_01260_amd.solver import Solver, SweError

    torch = torch_cuda
    pr = inputs_mod.c2_2d(64, "smooth", ny=40)
    with Solver.from_problem(pr) as s:
        st = torch.from_numpy(pr.state).cuda().contiguous()
        for al in ((float("nan"), 1.0), (1.0, float("nan")), (float("inf"), 1.0), (0.0, 1.0), (1.0, 0.0)):
            with pytest.raises(SweError):
                s.rhs(st, alpha=al)
        s.rhs(st, alpha=(5.0, 5.0))  # finite positive speeds are accepted
        s.sync()


@pytest.mark.parametrize("kind", ["dry", "nan"])
def test_bare_rhs_reports_bad_input(torch_cuda, inputs_mod, kind):
    """A right-hand side with given speeds skips the speed reduction, so the kernel itself flags a
    node with h <= 0 or a non-finite result: reported by swe_hweno_sync, and by the call itself
    with SWE_CHECK_DRY."""
    from paper_2208_01260_amd import _lib
    from paper_2208_01260_amd.solver import Solver, SweError

    torch = torch_cuda
    pr = inputs_mod.c2_2d(64, "smooth", ny=40)
    bad = pr.state.copy()
    if kind == "dry":
        bad[0, 17, 23] = pr.b[17, 23] - 0.05
        code = _lib.EDRY
    else:
        bad[4, 30, 50] = np.nan
        code = _lib.ENONFINITE
    st = torch.from_numpy(bad).cuda().contiguous()
    good = torch.from_numpy(pr.state).cuda().contiguous()
    with Solver.from_problem(pr) as s:
        s.rhs(good, alpha=(5.0, 5.0))
        s.sync()  # a good state reports nothing
        s.rhs(st, alpha=(5.0, 5.0))
        with pytest.raises(SweError) as e:
            s.sync()
        assert e.value.code == code
        s.sync()  # the flag was cleared
    with Solver.from_problem(pr, flags=_lib.CHECK_DRY) as s:
        s.rhs(good, alpha=(5.0, 5.0))
        with pytest.raises(SweError) as e:
            s.rhs(st, alpha=(5.0, 5.0))
        assert e.value.code == code
        s.step(good)  # a good step reports nothing even when checked
