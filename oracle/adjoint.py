"""Objective and finite-difference derivatives for checking the discrete
adjoint (test infrastructure only).

The quantity differentiated is a run of the oracle's own integrator (RK
bootstrap, then MRAB macrosteps; section "Multi-rate Adams-Bashforth
Integration") from initial states y0, and the objective written out from its
definition: the trapezoid-rule time integral, over one grid's own-step times
from the start of the macrosteps (step H / r_grid, halved at both ends), of a
weighted sum of the pressure p = (gamma - 1)(rho E - rho |u|^2 / 2) at listed
points.  Directional derivatives come from central differences with one
Richardson extrapolation, (4 D(h/2) - D(h)) / 3, D(h) = (f(x + h v) - f(x -
h v)) / (2 h), whose error is O(h^4) plus rounding.

Parity unpinned: the oracle holds no adjoint of its own; the library's
adjoint is checked against these directional derivatives of the oracle's
forward map (dot products <J^T w, v> = <w, J v>).
"""
from __future__ import annotations

from typing import Callable, List, Sequence

import numpy as np


def pressure(q: np.ndarray, gamma: float) -> np.ndarray:
    """p at every point of a state stored nv x npts."""
    dim = q.shape[0] - 2
    rho = q[0]
    ke = sum(q[1 + i] * q[1 + i] / rho for i in range(dim))
    return (gamma - 1.0) * (q[dim + 1] - 0.5 * ke)


def run_objective(osys, y0: Sequence[np.ndarray], nmacro: int, H: float, grid: int, pts, w):
    """(J, final states) of the oracle run from y0."""
    gamma = osys.params["gamma"]
    pts = np.asarray(pts, dtype=np.int64)
    w = np.asarray(w, dtype=np.float64)
    mr = osys.integrator(H)
    nv = osys.nv
    mr.bootstrap([np.asarray(y, dtype=np.float64).reshape(nv, -1).copy() for y in y0])
    rate = osys.wl.grids[grid].rate
    hg = H / rate
    last = nmacro * rate
    total = [0.0]
    count = [0]

    def term(y):
        i = count[0]
        tau = 0.5 * hg if (i == 0 or i == last) else hg
        total[0] += tau * float(np.dot(w, pressure(y.reshape(nv, -1), gamma)[pts]))
        count[0] += 1

    term(mr.y[grid])

    def observe(g, y):
        if g == grid:
            term(y)

    for _ in range(nmacro):
        mr.macrostep(observe)
    return total[0], [y.copy() for y in mr.y]


def richardson(f: Callable[[float], float], h: float) -> float:
    """d/de f(e) at e = 0: central differences at h and h/2, one Richardson
    step."""
    d1 = (f(h) - f(-h)) / (2.0 * h)
    d2 = (f(0.5 * h) - f(-0.5 * h)) / h
    return (4.0 * d2 - d1) / 3.0


def rhs_directional(osys, states: List[np.ndarray], v: List[np.ndarray], h: float) -> List[np.ndarray]:
    """J_rhs v of the coupled right-hand side (every grid, donor data at the
    same time) by Richardson-extrapolated central differences, per grid."""
    def f(e):
        st = [s + e * d for s, d in zip(states, v)]
        out = osys.rhs(st)
        return [out[g] for g in range(len(states))]

    fp, fm = f(h), f(-h)
    fp2, fm2 = f(0.5 * h), f(-0.5 * h)
    return [(4.0 * (a2 - b2) / h - (a - b) / (2.0 * h)) / 3.0 for a, b, a2, b2 in zip(fp, fm, fp2, fm2)]
