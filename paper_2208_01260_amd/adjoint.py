"""Differentiable runs of the 2D scheme: a torch.autograd.Function over the library's forward
run (swe_hweno_run_checkpointed, which keeps checkpoints) and its hand-written reverse
(swe_hweno_run_vjp_checkpointed).

The run is taken at a fixed dt with the Lax-Friedrichs speeds frozen (the map is then smooth).
The bottom enters through b alone: its slopes are b_x, b_y = D(b) by the library's fixed
fourth-order centred difference (swe_hweno_bottom_slopes), and the gradient with respect to b
adds the transpose of D applied to the slope adjoints.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import FIXED_ALPHA, FIXED_DT
from .solver import Solver, _dev


def _params(nx, ny, domain, bc, g=9.812, cfl=0.6, eps=1e-6):
    p = _lib.Params()
    p.dim, p.nx, p.ny = 2, int(nx), int(ny)
    p.x0, p.x1, p.y0, p.y1 = [float(v) for v in domain]
    p.g, p.cfl, p.eps = g, cfl, eps
    p.bc_x, p.bc_y = int(bc[0]), int(bc[1])
    return p


def bottom_slopes(b, domain, bc):
    """(b_x, b_y) of a (ny, nx) float64 CUDA tensor by the library's centred difference."""
    ny, nx = b.shape
    p = _params(nx, ny, domain, bc)
    bx, by = torch.empty_like(b), torch.empty_like(b)
    _lib.check(_lib.lib().swe_hweno_bottom_slopes(ctypes.byref(p), _dev(b, "b"), bx.data_ptr(), by.data_ptr(),
                                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
               "swe_hweno_bottom_slopes")
    return bx, by


def bottom_slopes_vjp(bxbar, bybar, bbar, domain, bc):
    """bbar += D^T (bxbar, bybar) (in place)."""
    ny, nx = bbar.shape
    p = _params(nx, ny, domain, bc)
    _lib.check(_lib.lib().swe_hweno_bottom_slopes_vjp(ctypes.byref(p), _dev(bxbar, "bxbar", shape=(ny, nx)),
                                                      _dev(bybar, "bybar", shape=(ny, nx)), _dev(bbar, "bbar"),
                                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
               "swe_hweno_bottom_slopes_vjp")
    return bbar


class SWERun(torch.autograd.Function):
    """state_T = run(state0, b): nsteps steps at dt with frozen alpha = (ax, ay)."""

    @staticmethod
    def forward(ctx, state0, b, domain, bc, nsteps, dt, alpha, checkpoint_every, g, cfl, eps):
        bx, by = bottom_slopes(b, domain, bc)
        ny, nx = b.shape
        s = Solver(2, nx, ny, domain, b, bx, by, bc=bc, g=g, cfl=cfl, eps=eps, flags=FIXED_DT | FIXED_ALPHA,
                   fixed_dt=dt, alpha=alpha)
        st = state0.detach().clone()
        s.run_checkpointed(st, nsteps, checkpoint_every)
        ctx.solver, ctx.nsteps, ctx.ck, ctx.domain, ctx.bc = s, nsteps, checkpoint_every, domain, bc
        return st

    @staticmethod
    def backward(ctx, grad_out):
        s = ctx.solver
        sbar0, bb, bxb, byb = s.run_vjp_checkpointed(ctx.nsteps, grad_out.contiguous(), ctx.ck)
        bottom_slopes_vjp(bxb, byb, bb, ctx.domain, ctx.bc)
        s.close()
        return sbar0, bb, None, None, None, None, None, None, None, None, None


def run(state0, b, domain, bc, nsteps, dt, alpha, checkpoint_every=10, g=9.812, cfl=0.6, eps=1e-6):
    """Differentiable run: gradients flow to state0 (9, ny, nx) and b (ny, nx)."""
    return SWERun.apply(state0, b, tuple(domain), tuple(bc), int(nsteps), float(dt), tuple(alpha),
                        int(checkpoint_every), g, cfl, eps)
