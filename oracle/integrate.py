"""Time integration for the oracle: RK bootstrap, single-rate AB, multi-rate AB.

Part of the test oracle (test infrastructure only).

Paper: section "Adams-Bashforth Integration" (eq. ab_general; third-order Heun
RK bootstraps third-order AB, classic fourth-order RK bootstraps fourth-order
AB), section "Extended-History Adams-Bashforth Schemes" (m > n history values),
and section "Multi-rate Adams-Bashforth Integration": the fastest-first scheme
without re-extrapolation, Steps 1-7, generalised to integer step ratios and to
more than two rates (the paper states the approach extends to any number).

Readings: a level with rate r takes r steps of H/r per macrostep H; the
micro-step is delta = H / r_max.  At micro-time k (k = 1..r_max) every level
whose own step ends at k advances from its last own state with its own-step
coefficients; every other level is represented by its extrapolant integrated
from its last own time (no re-extrapolation, whole grid); the levels whose step
ends at k evaluate their right-hand side and push it into their history.
Bootstrap: single-rate RK at delta for (m-1)*r_max steps, keeping the first
stage value F(y_n) at each level's history node times.

Summation order of every history combination: y, then oldest to newest
(acc = acc + c_j * F_j), each product and sum rounded separately.
"""
from __future__ import annotations

from fractions import Fraction as Fr
from typing import Callable, Dict, List

import numpy as np

from .coeffs import ab_coefficients


def combine(y: np.ndarray, c: List[float], hist: List[np.ndarray]) -> np.ndarray:
    acc = y.copy()
    for cj, Fj in zip(c, hist):
        acc = acc + cj * Fj
    return acc


class MRAB:
    """rhs(states, which) -> {g: F_g} for g in which, states = list of arrays."""

    def __init__(self, rhs: Callable, rates: List[int], order: int, hist_len: int, H: float):
        self.rhs = rhs
        self.rates = list(rates)
        self.order, self.m = order, hist_len
        self.r_max = max(rates)
        for r in rates:
            if r < 1 or self.r_max % r:
                raise ValueError("every rate must divide the largest rate")
        self.H = H
        self.delta = H / self.r_max
        self.c_own, self.beta = [], []
        for r in rates:
            Hg = H / r
            self.c_own.append([float(a) * Hg for a in ab_coefficients(order, hist_len, Fr(1))])
            rows = {}
            for jp in range(1, self.r_max // r):
                tau = Fr(jp * r, self.r_max)
                rows[jp] = [float(a) * Hg for a in ab_coefficients(order, hist_len, tau)]
            self.beta.append(rows)
        self.y: List[np.ndarray] = []
        self.hist: List[List[np.ndarray]] = []
        self.t = 0.0

    # ---------------------------------------------------------------- start
    def bootstrap(self, y0: List[np.ndarray], t0: float = 0.0):
        G = len(y0)
        d = self.delta
        nsteps = (self.m - 1) * self.r_max
        keep = [set(nsteps - j * (self.r_max // r) for j in range(self.m)) for r in self.rates]
        hist = [[] for _ in range(G)]
        y = [a.copy() for a in y0]
        allg = list(range(G))
        for n in range(nsteps + 1):
            k1 = self.rhs(y, allg)
            for g in range(G):
                if n in keep[g]:
                    hist[g].append(k1[g])
            if n == nsteps:
                break
            if self.order <= 3:
                k2 = self.rhs([y[g] + (d / 3.0) * k1[g] for g in allg], allg)
                k3 = self.rhs([y[g] + (2.0 * d / 3.0) * k2[g] for g in allg], allg)
                y = [y[g] + (d / 4.0) * (k1[g] + 3.0 * k3[g]) for g in allg]
            else:
                k2 = self.rhs([y[g] + (d / 2.0) * k1[g] for g in allg], allg)
                k3 = self.rhs([y[g] + (d / 2.0) * k2[g] for g in allg], allg)
                k4 = self.rhs([y[g] + d * k3[g] for g in allg], allg)
                y = [y[g] + (d / 6.0) * (k1[g] + 2.0 * k2[g] + 2.0 * k3[g] + k4[g]) for g in allg]
        self.y = y
        self.hist = hist
        self.t = t0 + nsteps * d

    def set_history(self, y: List[np.ndarray], hist: List[List[np.ndarray]], t: float):
        self.y = [a.copy() for a in y]
        self.hist = [[h.copy() for h in hs] for hs in hist]
        self.t = t

    # ------------------------------------------------------------ macrostep
    def macrostep(self, observe=None):
        """One macrostep; observe(g, y), when given, sees every level's state
        right after each of its own steps."""
        G = len(self.y)
        for k in range(1, self.r_max + 1):
            per = [self.r_max // r for r in self.rates]
            ends = [k % per[g] == 0 for g in range(G)]
            for g in range(G):
                if ends[g]:
                    self.y[g] = combine(self.y[g], self.c_own[g], self.hist[g])
                    if observe is not None:
                        observe(g, self.y[g])
            states = []
            for g in range(G):
                if ends[g]:
                    states.append(self.y[g])
                else:
                    states.append(combine(self.y[g], self.beta[g][k % per[g]], self.hist[g]))
            which = [g for g in range(G) if ends[g]]
            F = self.rhs(states, which)
            for g in which:
                self.hist[g].pop(0)
                self.hist[g].append(F[g])
        self.t += self.H


def srab_steps(rhs: Callable, y: List[np.ndarray], hist: List[List[np.ndarray]],
               c: List[float], nsteps: int):
    """Independent single-rate AB loop (every level at the same step)."""
    y = [a.copy() for a in y]
    hist = [[h.copy() for h in hs] for hs in hist]
    G = len(y)
    for _ in range(nsteps):
        y = [combine(y[g], c, hist[g]) for g in range(G)]
        F = rhs(y, list(range(G)))
        for g in range(G):
            hist[g] = hist[g][1:] + [F[g]]
    return y, hist


def rk4_steps(rhs: Callable, y: List[np.ndarray], h: float, nsteps: int) -> List[np.ndarray]:
    """Classic fourth-order Runge-Kutta, every level at step h (the reference
    integrator of section "Multi-Rate Adams-Bashforth Accuracy and
    Convergence")."""
    G = len(y)
    allg = list(range(G))
    y = [a.copy() for a in y]
    for _ in range(nsteps):
        k1 = rhs(y, allg)
        k2 = rhs([y[g] + (h / 2.0) * k1[g] for g in allg], allg)
        k3 = rhs([y[g] + (h / 2.0) * k2[g] for g in allg], allg)
        k4 = rhs([y[g] + h * k3[g] for g in allg], allg)
        y = [y[g] + (h / 6.0) * (k1[g] + 2.0 * k2[g] + 2.0 * k3[g] + k4[g]) for g in allg]
    return y
