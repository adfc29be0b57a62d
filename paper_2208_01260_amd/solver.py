"""Thin Python front end of the HIP solver: torch tensors in, the C ABI underneath.

PyTorch provides device memory and streams only. A state is a contiguous CUDA tensor of shape
(4, nx) in 1D (eta, m, H, M) or (9, ny, nx) in 2D (eta, m, w, H1, M1, W1, H2, M2, W2), float64,
or float32 for a single-precision solver (dtype=torch.float32, the library's _f32 entry points).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import BC_PERIODIC, BC_REFLECTIVE, FIXED_ALPHA, FIXED_DT, NO_LIMITER, SweError  # noqa: F401


def _dev(t: torch.Tensor, name: str, dtype=torch.float64, shape=None) -> int:
    """Device pointer of a contiguous CUDA tensor of the given dtype (and shape, when given: the
    library reads and writes exactly that many elements, so a wrong shape is refused here)."""
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != dtype:
        raise TypeError(f"{name} must be a {dtype} CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}")
    return t.data_ptr()


class Solver:
    """One solver context (swe_hweno_init ... swe_hweno_destroy) on the current CUDA stream."""

    def __init__(self, dim, nx, ny, domain, b, bx, by=None, bc=(BC_PERIODIC, BC_PERIODIC), g=9.812, cfl=0.6,
                 eps=1e-6, flags=0, fixed_dt=0.0, alpha=(0.0, 0.0), stream=None, dtype=torch.float64):
        L = _lib.lib()
        if dtype not in (torch.float64, torch.float32):
            raise TypeError("dtype must be torch.float64 or torch.float32")
        self.dtype = dtype
        sfx = "_f32" if dtype == torch.float32 else ""
        self._fn = {k: getattr(L, f"swe_hweno_{k}{sfx}") for k in ("init", "rhs", "limit", "alpha", "step", "run")}
        self.dim, self.nx, self.ny = dim, nx, (ny if dim == 2 else 1)
        self.nf = 9 if dim == 2 else 4
        self.shape = (9, self.ny, nx) if dim == 2 else (4, nx)
        p = _lib.Params()
        p.dim, p.nx, p.ny = dim, nx, self.ny
        p.x0, p.x1, p.y0, p.y1 = [float(v) for v in domain]
        p.g, p.cfl, p.eps = g, cfl, eps
        p.bc_x, p.bc_y, p.flags = int(bc[0]), int(bc[1]), int(flags)
        p.fixed_dt, p.alpha_x, p.alpha_y = float(fixed_dt), float(alpha[0]), float(alpha[1])
        self.params = p
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        keep = [b, bx] + ([by] if dim == 2 else [])
        ptrs = [_dev(t, n, dtype) for t, n in zip(keep, ("b", "bx", "by"))]
        for t in keep:
            if t.numel() != nx * self.ny:
                raise ValueError("bottom planes must have nx*ny elements")
        ctx = ctypes.c_void_p()
        _lib.check(self._fn["init"](ctypes.byref(p), ptrs[0], ptrs[1], ptrs[2] if dim == 2 else None,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx)), "swe_hweno_init")
        self._ctx = ctx
        self._L = L

    @classmethod
    def from_problem(cls, prob, device="cuda", dtype=torch.float64, **kw):
        """Build from a paper_2208_01260_amd.inputs.Problem (bottom copied to the device)."""
        t = lambda a: torch.from_numpy(a).to(device=device, dtype=dtype).contiguous()
        d = dict(bc=prob.bc, g=prob.g, cfl=prob.cfl, eps=prob.eps)
        d.update(kw)
        return cls(prob.dim, prob.nx, prob.ny, prob.domain, t(prob.b), t(prob.bx),
                   t(prob.by) if prob.dim == 2 else None, dtype=dtype, **d)

    def _state(self, s, name="state"):
        ptr = _dev(s, name, self.dtype)
        if tuple(s.shape) != self.shape:
            raise ValueError(f"{name} must have shape {self.shape}")
        return ptr

    def rhs(self, state, out=None, alpha=None):
        out = torch.empty_like(state) if out is None else out
        ax, ay = (-1.0, -1.0) if alpha is None else (float(alpha[0]), float(alpha[1]))
        _lib.check(self._fn["rhs"](self._ctx, self._state(state), self._state(out, "out"), ax, ay), "swe_hweno_rhs")
        return out

    def limit(self, state, out=None):
        nd = 6 if self.dim == 2 else 2
        shape = (nd,) + self.shape[1:]
        out = torch.empty(shape, dtype=self.dtype, device=state.device) if out is None else out
        _lib.check(self._fn["limit"](self._ctx, self._state(state), _dev(out, "out", self.dtype, shape)),
                   "swe_hweno_limit")
        return out

    def alpha(self, state):
        a = (ctypes.c_double * 2)()
        _lib.check(self._fn["alpha"](self._ctx, self._state(state), a), "swe_hweno_alpha")
        return a[0], a[1]

    def step(self, state, dt=0.0, sync=False):
        used = ctypes.c_double()
        _lib.check(self._fn["step"](self._ctx, self._state(state), float(dt), ctypes.byref(used) if sync else None),
                   "swe_hweno_step")
        return used.value if sync else None

    def run(self, state, nsteps=0, t_end=0.0):
        t, k = ctypes.c_double(), ctypes.c_int()
        _lib.check(self._fn["run"](self._ctx, self._state(state), int(nsteps), float(t_end), ctypes.byref(t),
                                   ctypes.byref(k)), "swe_hweno_run")
        return t.value, k.value

    def set_timing(self, on=True):
        """Event-time every fused stage kernel (direct launches instead of graph replay)."""
        _lib.check(self._L.swe_hweno_set_timing(self._ctx, 1 if on else 0), "swe_hweno_set_timing")

    def get_timing(self):
        """{'rhs'|'stage1'|'stage2'|'stage3': (total ms, launches)} since timing was turned on."""
        ms, n = (ctypes.c_double * 4)(), (ctypes.c_longlong * 4)()
        _lib.check(self._L.swe_hweno_get_timing(self._ctx, ms, n), "swe_hweno_get_timing")
        return {k: (ms[i], n[i]) for i, k in enumerate(("rhs", "stage1", "stage2", "stage3"))}

    def tile(self):
        """(output columns per wavefront, rows per wavefront march) of this context."""
        c, r = ctypes.c_int(), ctypes.c_int()
        _lib.check(self._L.swe_hweno_ctx_tile(self._ctx, ctypes.byref(c), ctypes.byref(r)), "swe_hweno_ctx_tile")
        return c.value, r.value

    def sync(self):
        _lib.check(self._L.swe_hweno_sync(self._ctx), "swe_hweno_sync")

    # ------------------------------------------------------------------ reverse mode (2D FP64)
    def _planes(self, like=None):
        return torch.empty((self.ny, self.nx), dtype=torch.float64, device="cuda") if like is None else like

    def rhs_vjp(self, state, rbar, alpha):
        """(sbar, bbar, bxbar, bybar) = rbar^T d R(state) / d(state, b, bx, by), alpha frozen."""
        sbar = torch.empty_like(state)
        bb, bxb, byb = self._planes(), self._planes(), self._planes()
        _lib.check(self._L.swe_hweno_rhs_vjp(self._ctx, self._state(state), float(alpha[0]), float(alpha[1]),
                                             self._state(rbar, "rbar"), sbar.data_ptr(), bb.data_ptr(),
                                             bxb.data_ptr(), byb.data_ptr()), "swe_hweno_rhs_vjp")
        return sbar, bb, bxb, byb

    def limit_vjp(self, state, dmbar):
        """(sbar, bbar) = dmbar^T d Lim(state) / d(state, b)."""
        sbar = torch.empty_like(state)
        bb = self._planes()
        dshape = (6, self.ny, self.nx)
        _lib.check(self._L.swe_hweno_limit_vjp(self._ctx, self._state(state), _dev(dmbar, "dmbar", shape=dshape),
                                               sbar.data_ptr(),
                                               bb.data_ptr()), "swe_hweno_limit_vjp")
        return sbar, bb

    def run_checkpointed(self, state, nsteps, checkpoint_every=10):
        """nsteps fixed-dt, frozen-alpha steps of state in place, keeping checkpoints for
        run_vjp_checkpointed."""
        _lib.check(self._L.swe_hweno_run_checkpointed(self._ctx, self._state(state), int(nsteps),
                                                      int(checkpoint_every)), "swe_hweno_run_checkpointed")

    def run_vjp_checkpointed(self, nsteps, sbar_T, checkpoint_every=10):
        """Reverse of the last run_checkpointed: (sbar_0, bbar, bxbar, bybar)."""
        sbar0 = torch.empty_like(sbar_T)
        bb, bxb, byb = self._planes(), self._planes(), self._planes()
        _lib.check(self._L.swe_hweno_run_vjp_checkpointed(self._ctx, int(nsteps), int(checkpoint_every),
                                                          self._state(sbar_T, "sbar_T"), sbar0.data_ptr(),
                                                          bb.data_ptr(), bxb.data_ptr(), byb.data_ptr()),
                   "swe_hweno_run_vjp_checkpointed")
        return sbar0, bb, bxb, byb

    def run_vjp(self, state0, nsteps, sbar_T, checkpoint_every=10):
        """Reverse of `nsteps` fixed-dt, frozen-alpha steps from state0: returns
        (sbar_0, bbar, bxbar, bybar) for the adjoint sbar_T of the final state."""
        sbar0 = torch.empty_like(state0)
        bb, bxb, byb = self._planes(), self._planes(), self._planes()
        _lib.check(self._L.swe_hweno_run_vjp(self._ctx, self._state(state0), int(nsteps), int(checkpoint_every),
                                             self._state(sbar_T, "sbar_T"), sbar0.data_ptr(), bb.data_ptr(),
                                             bxb.data_ptr(), byb.data_ptr()), "swe_hweno_run_vjp")
        return sbar0, bb, bxb, byb

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._L.swe_hweno_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def tile():
    c, r = ctypes.c_int(), ctypes.c_int()
    _lib.check(_lib.lib().swe_hweno_tile(ctypes.byref(c), ctypes.byref(r)))
    return c.value, r.value


class Batch:
    """Many independent 2D instances advanced together (swe_hweno_batch_*) on the current CUDA
    stream. `problems` are paper_2208_01260_amd.inputs.Problem objects sharing g, cfl and eps; each
    one's state is copied to the device into `self.states[i]` (shape (9, ny, nx)), unless `states`
    gives the device tensors to advance in place. The bottoms are copied by the library."""

    def __init__(self, problems, states=None, flags=0, fixed_dt=0.0, alpha=(0.0, 0.0), device="cuda", stream=None):
        L = _lib.lib()
        if not problems:
            raise ValueError("a batch needs at least one instance")
        g, cfl, eps = problems[0].g, problems[0].cfl, problems[0].eps
        t = lambda a: torch.from_numpy(a).to(device=device, dtype=torch.float64).contiguous()
        self.states = list(states) if states is not None else [t(pr.state) for pr in problems]
        arr = (_lib.Instance * len(problems))()
        keep = []
        for i, pr in enumerate(problems):
            if pr.dim != 2 or (pr.g, pr.cfl, pr.eps) != (g, cfl, eps):
                raise ValueError("batched instances are 2D and share g, cfl and eps")
            st = self.states[i]
            ptr = _dev(st, f"states[{i}]")
            if tuple(st.shape) != (9, pr.ny, pr.nx):
                raise ValueError(f"states[{i}] must have shape {(9, pr.ny, pr.nx)}")
            b, bx, by = t(pr.b), t(pr.bx), t(pr.by)
            for a, nm in ((b, "b"), (bx, "bx"), (by, "by")):
                if tuple(a.shape) != (pr.ny, pr.nx):
                    raise ValueError(f"instance {i}: {nm} must have shape {(pr.ny, pr.nx)}")
            keep += [b, bx, by]
            it = arr[i]
            it.nx, it.ny = pr.nx, pr.ny
            it.x0, it.x1, it.y0, it.y1 = [float(v) for v in pr.domain]
            it.bc_x, it.bc_y = int(pr.bc[0]), int(pr.bc[1])
            it.b, it.bx, it.by, it.state = b.data_ptr(), bx.data_ptr(), by.data_ptr(), ptr
        p = _lib.Params()
        p.dim, p.nx, p.ny = 2, 4, 4
        p.x0, p.x1, p.y0, p.y1 = 0.0, 1.0, 0.0, 1.0
        p.g, p.cfl, p.eps, p.flags = g, cfl, eps, int(flags)
        p.fixed_dt, p.alpha_x, p.alpha_y = float(fixed_dt), float(alpha[0]), float(alpha[1])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _lib.check(L.swe_hweno_batch_init(ctypes.byref(p), arr, len(problems), ctypes.c_void_p(self.stream.cuda_stream),
                                          ctypes.byref(h)), "swe_hweno_batch_init")
        self._h, self._L, self.count = h, L, len(problems)
        self.cells = sum(pr.nx * pr.ny for pr in problems)

    def run(self, nsteps):
        """nsteps steps of every instance; returns the time each advanced."""
        t = (ctypes.c_double * self.count)()
        _lib.check(self._L.swe_hweno_batch_run(self._h, int(nsteps), t), "swe_hweno_batch_run")
        return list(t)

    def set_rows(self, rows):
        _lib.check(self._L.swe_hweno_batch_set_rows(self._h, int(rows)), "swe_hweno_batch_set_rows")

    def autotune(self):
        """Rows per march for this batch: timed, or taken from the process-wide cache of its size class."""
        r = ctypes.c_int()
        _lib.check(self._L.swe_hweno_batch_autotune(self._h, ctypes.byref(r)), "swe_hweno_batch_autotune")
        return r.value

    @staticmethod
    def tune_cache_size():
        return _lib.lib().swe_hweno_batch_tune_cache_size()

    @staticmethod
    def tune_cache_clear():
        _lib.lib().swe_hweno_batch_tune_cache_clear()

    def sync(self):
        _lib.check(self._L.swe_hweno_batch_sync(self._h), "swe_hweno_batch_sync")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.swe_hweno_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
