"""The allocation-free step (swe_hweno_step_noalloc) against the context-based step
(swe_hweno_step) on the same inputs, through the C ABI: two calls in a row on one GPU, the second
on a smaller grid, then a 1D grid. Both run the same kernels with the same tiles, so the results
are bitwise equal; the scratch array that the second call reuses must not leak the first call's
contents into it."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _run_pair(pr, dt, want_dt):
    import torch

    from paper_2208_01260_amd import _lib
    from paper_2208_01260_amd.solver import Solver

    L = _lib.lib()
    dev = torch.device("cuda:0")
    st0 = torch.from_numpy(pr.state).to(dev).contiguous()
    with Solver.from_problem(pr, device=dev) as s:
        ref = st0.clone()
        dref = s.step(ref, dt=dt, sync=True)
        p = s.params
    t = lambda a: torch.from_numpy(a).to(dev).contiguous()
    b, bx = t(pr.b), t(pr.bx)
    by = t(pr.by) if pr.dim == 2 else None
    got = st0.clone()
    used = ctypes.c_double(-1.0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.swe_hweno_step_noalloc(ctypes.byref(p), got.data_ptr(), b.data_ptr(), bx.data_ptr(),
                                  by.data_ptr() if by is not None else None, float(dt), stream,
                                  ctypes.byref(used) if want_dt else None)
    assert rc == 0, _lib.strerror(rc)
    torch.cuda.synchronize()
    g, r = got.cpu().numpy(), ref.cpu().numpy()
    print(f"{pr.name} {pr.nx}x{pr.ny}: max |noalloc - step| = {np.abs(g - r).max():.3e}", flush=True)
    assert np.array_equal(g, r)
    assert not np.array_equal(g, pr.state)  # the step did something
    if want_dt:
        assert used.value == dref


def test_noalloc_step_matches_context_step_twice_then_smaller_and_1d():
    from paper_2208_01260_amd import inputs

    # first call: 2D 200 x 150 with walls, CFL step, dt reported (synchronising form)
    _run_pair(inputs.c2_2d(200, "smooth", ny=150), 0.0, True)
    # second call on the same GPU: a smaller periodic grid, a given dt, no synchronisation
    pr = inputs.c2_2d(96, "smooth", ny=70)
    pr.bc = (0, 0)
    _run_pair(pr, 2e-4, False)
    # 1D
    _run_pair(inputs.c1_1d(200), 0.0, True)


def test_noalloc_rejects_grids_beyond_the_array():
    from paper_2208_01260_amd import _lib

    L = _lib.lib()
    cap = L.swe_hweno_noalloc_capacity()
    p = _lib.Params()
    p.dim, p.nx, p.ny = 2, 419, 419
    p.x0, p.x1, p.y0, p.y1 = 0.0, 1.0, 0.0, 1.0
    p.g, p.cfl, p.eps = 9.812, 0.6, 1e-6
    assert 256 + 24 * 419 * 419 * 8 > cap
    fake = ctypes.c_void_p(0x1000)
    assert L.swe_hweno_step_noalloc(ctypes.byref(p), fake, fake, fake, fake, 0.0, None, None) == -1
