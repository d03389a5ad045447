"""Discrete adjoint of a run (RK bootstrap + MRAB macrosteps) on the GPU.

The library differentiates its own forward pass: from initial states y0 it
bootstraps the histories (single-rate RK at the micro-step), takes nmacro
MRAB macrosteps at the context's fixed macrostep H, and accumulates

    J = sum_i tau_i sum_k w_k p(q_grid(pts_k, t_i)),

the trapezoid-rule time integral over the objective grid's own-step times of
a weighted pressure sum at listed points (with w_k = n_x ds on a wall, the
time-integrated pressure force along x).  Gradients come from hand-written
adjoint kernels run in reverse order, with the macrosteps reversed under a
binomial checkpointing schedule (nsnap snapshots of the states and AB
histories).  Method: section "Multi-rate Adams-Bashforth Integration" (the
forward schedule being reversed) and section "Adams-Bashforth Integration"
(the bootstrap and the history combinations).

``MRABRun`` wraps a run as a ``torch.autograd.Function`` of the initial
states: it returns J and the final states; its backward pass is one call of
the library's reverse sweep (which reruns the forward pass under the
checkpointing schedule).
"""
from __future__ import annotations

from ctypes import POINTER, byref, c_double, c_int64, c_size_t, c_void_p
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from .system import System


def _ptrs(ts: Sequence[Optional[torch.Tensor]]):
    return (c_void_p * len(ts))(*[t.data_ptr() if t is not None else None for t in ts])


class Adjoint:
    """Adjoint workspace of a System (2D) with nsnap snapshot slots."""

    def __init__(self, sysg: System, nsnap: int = 20):
        self.s = sysg
        self.lib = sysg.lib
        self.nsnap = nsnap
        nbytes = c_size_t()
        sysg._check(self.lib.mr_adj_workspace_size(sysg.ctx, nsnap, byref(nbytes)), "mr_adj_workspace_size")
        self.ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=sysg.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        sysg._check(self.lib.mr_adj_bind_workspace(sysg.ctx, c_void_p(base + off), c_size_t(nbytes.value)),
                    "mr_adj_bind_workspace")
        self.nbytes = int(nbytes.value)

    def set_objective(self, grid: int, pts, w) -> None:
        pts = np.ascontiguousarray(pts, dtype=np.int64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        self.s._check(self.lib.mr_adj_set_objective(self.s.ctx, grid, len(pts), pts.ctypes.data_as(POINTER(c_int64)),
                                                    w.ctypes.data_as(POINTER(c_double))), "mr_adj_set_objective")

    def _states(self, ys) -> List[torch.Tensor]:
        return [self.s._dev(y).reshape(self.s.nv, -1) for y in ys]

    def rhs_vjp(self, states, lamF) -> List[torch.Tensor]:
        """(d rhs / d q)^T lamF for the coupled right-hand side at states."""
        qs, ls = self._states(states), self._states(lamF)
        outs = [torch.empty_like(q) for q in qs]
        self.s._check(self.lib.mr_adj_rhs(self.s.ctx, _ptrs(qs), _ptrs(ls), _ptrs(outs)), "mr_adj_rhs")
        self._alive = (qs, ls, outs)
        return outs

    def forward(self, nmacro: int, y0):
        """(J, final states) of the run from y0."""
        ys = self._states(y0)
        outs = [torch.empty_like(y) for y in ys]
        J = c_double()
        self.s._check(self.lib.mr_adj_forward(self.s.ctx, nmacro, _ptrs(ys), _ptrs(outs), byref(J)), "mr_adj_forward")
        self._alive = (ys, outs)
        return J.value, outs

    def gradient(self, nmacro: int, y0, lamN=None, jscale: float = 1.0):
        """(J, dL/dy0 per grid, forward macrosteps run) for L = jscale J +
        sum_g <lamN[g], yN[g]>."""
        ys = self._states(y0)
        ln = [None] * len(ys) if lamN is None else [None if l is None else self.s._dev(l).reshape(self.s.nv, -1)
                                                     for l in lamN]
        grads = [torch.empty_like(y) for y in ys]
        J = c_double()
        nf = c_int64()
        self.s._check(self.lib.mr_adj_gradient(self.s.ctx, nmacro, _ptrs(ys), _ptrs(ln), jscale, _ptrs(grads),
                                               byref(J), byref(nf)), "mr_adj_gradient")
        self._alive = (ys, ln, grads)
        self.last_nfwd = nf.value
        return J.value, grads, nf.value


def schedule_cost(nmacro: int, nsnap: int) -> int:
    """Forward macrosteps the checkpointed reversal of nmacro macrosteps
    recomputes with nsnap snapshot slots (slot 0 holding the start)."""
    lib = _lib.load()
    n = c_int64()
    _lib.check(lib.mr_adj_schedule(nmacro, nsnap, byref(n)), None, "mr_adj_schedule")
    return n.value


def wall_objective(grid) -> tuple:
    """Points and weights n_x ds of the first radial line (the wall) of a 2D
    O-mesh grid: the outward normal of the body is the radial direction at
    each wall point, ds = r dtheta (uniform in theta)."""
    nt = grid.n[0]
    x, y = grid.coords[0][:nt], grid.coords[1][:nt]
    r = np.hypot(x, y)
    return np.arange(nt, dtype=np.int64), (x / r) * r * (2.0 * np.pi / nt)


class MRABRun(torch.autograd.Function):
    """J, *yN = MRABRun.apply(adj, nmacro, *y0): the run from initial states
    y0 (one tensor per grid); the gradient is the library's adjoint."""

    @staticmethod
    def forward(ctx, adj: Adjoint, nmacro: int, *y0):
        J, outs = adj.forward(nmacro, y0)
        ctx.adj, ctx.nmacro = adj, nmacro
        ctx.shapes = [y.shape for y in y0]
        ctx.save_for_backward(*[y.detach() for y in y0])
        Jt = torch.tensor(J, dtype=torch.float64, device=adj.s.device)
        return (Jt, *[o.reshape(s) for o, s in zip(outs, ctx.shapes)])

    @staticmethod
    def backward(ctx, gJ, *gys):
        y0 = ctx.saved_tensors
        lamN = [None if g is None else g.reshape(ctx.adj.s.nv, -1) for g in gys]
        jscale = 0.0 if gJ is None else float(gJ)
        _, grads, _ = ctx.adj.gradient(ctx.nmacro, y0, lamN, jscale)
        return (None, None, *[g.reshape(s) for g, s in zip(grads, ctx.shapes)])
