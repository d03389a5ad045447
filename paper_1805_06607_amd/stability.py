"""Stability tooling on the GPU path: step matrices of the MRAB integrator
and approximate stability regions of the single-rate schemes.

Step matrices (section "Procedure for Determining Discrete Stability"): the
integrator state is every grid's state and its m right-hand-side history
values; one step of the integrator is one MRAB macrostep H.  Columns are
finite differences (perturbation eps of one state entry, 1e-7 in the paper)
of one macrostep run by the library's kernels, set through mr_set_state /
mr_set_history / mr_mrab_resume.  The integrator is deemed stable at H when
the spectral radius is at most 1; the largest stable H is searched by
bisection (to 1e-4 in the paper).  Dense matrices suit small systems; for
larger ones the spectral radius comes from Arnoldi iterations on the
finite-difference map (scipy), each product one GPU macrostep.

Stability regions (Appendix "Plotting Approximate Stability Regions"): the
boundary locus of an AB scheme with coefficients a_j (oldest first, unit
step) is z(theta) = (w^m - w^(m-1)) / sum_j a_j w^j, w = e^{i theta}; for
classic RK4 the curve |1 + z + z^2/2 + z^3/6 + z^4/24| = 1 is traced along
rays.  Regions can be normalised by right-hand-side evaluations per step
(RK4: 4, AB: 1), as the paper plots them.
"""
from __future__ import annotations

from typing import Callable, List, Optional

import numpy as np
import torch

from .system import System, ab_coeffs


# ----------------------------------------------------------------- regions
def ab_boundary_locus(order: int, hist_len: int, ntheta: int = 500) -> np.ndarray:
    """Boundary locus z(theta) of AB_order with hist_len history values (one
    right-hand-side evaluation per step, so already normalised)."""
    a = np.asarray(ab_coeffs(order, hist_len, 1.0))
    m = hist_len
    th = np.linspace(0.0, 2.0 * np.pi, ntheta, endpoint=False)
    w = np.exp(1j * th)
    num = w ** m - w ** (m - 1)
    den = sum(a[j] * w ** j for j in range(m))
    return num / den


def rk4_boundary(ntheta: int = 500, normalise: bool = True, tol: float = 1e-12) -> np.ndarray:
    """Points of |R_RK4(z)| = 1 along rays from z = -1 (inside the region),
    each by bisection; normalised by the 4 evaluations per step."""
    th = np.linspace(0.0, 2.0 * np.pi, ntheta, endpoint=False)

    def R(z):
        return abs(1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24)

    out = np.empty(ntheta, dtype=complex)
    for i, t in enumerate(th):
        d = np.exp(1j * t)
        lo, hi = 0.0, 6.0
        while hi - lo > tol:
            mid = 0.5 * (lo + hi)
            if R(-1.0 + mid * d) <= 1.0:
                lo = mid
            else:
                hi = mid
        out[i] = -1.0 + lo * d
    return out / 4.0 if normalise else out


def real_axis_reach(locus: np.ndarray) -> float:
    """Extent of a region along the negative real axis: the crossing of its
    boundary curve with the negative real axis nearest the origin (the
    curves of extended-history schemes cross it again further out, around
    unstable lobes)."""
    z = np.asarray(locus)
    best = np.inf
    for a, b in zip(z, np.roll(z, -1)):
        if a.imag == 0.0 and a.real < -1e-12:
            x = a.real
        elif a.imag * b.imag < 0:
            x = a.real - a.imag * (b.real - a.real) / (b.imag - a.imag)
        else:
            continue
        if x < -1e-12:
            best = min(best, -x)
    return float(best)


def imag_axis_reach(locus: np.ndarray) -> float:
    """Largest |Im z| where the boundary curve crosses the imaginary axis."""
    z = np.asarray(locus)
    best = 0.0
    for a, b in zip(z, np.roll(z, -1)):
        if a.real * b.real < 0:
            y = a.imag - a.real * (b.imag - a.imag) / (b.real - a.real)
            best = max(best, abs(y))
    return float(best)


# ------------------------------------------------------------ step matrices
class StepMap:
    """One MRAB macrostep of a System as a map on its integrator state."""

    def __init__(self, sysg: System):
        self.s = sysg
        self.nv = sysg.nv
        self.m = sysg.wl.params["hist_len"]
        self.sizes = [sysg.npts(g) * self.nv for g in range(sysg.ngrids)]
        self.n = sum(n * (1 + self.m) for n in self.sizes)

    def pack(self) -> np.ndarray:
        """Current integrator state: per grid the state, then its history
        values oldest first."""
        parts = []
        for g in range(self.s.ngrids):
            parts.append(self.s.state(g).reshape(-1))
            parts.extend(self.s.history(g, j).reshape(-1) for j in range(self.m))
        return torch.cat(parts).cpu().numpy()

    def load(self, x: np.ndarray, t: float = 0.0):
        xt = torch.as_tensor(x, dtype=torch.float64, device=self.s.device)
        off, states = 0, []
        for g, n in enumerate(self.sizes):
            states.append(xt[off:off + n])
            off += n
            for j in range(self.m):
                self.s.set_history(g, j, xt[off:off + n])
                off += n
        self.s.set_states(states)
        self.s.resume(t)

    def apply(self, x: np.ndarray) -> np.ndarray:
        self.load(x)
        self.s.macrostep(1)
        return self.pack()

    def columns(self, x0: np.ndarray, eps: float = 1e-7, cols: Optional[List[int]] = None) -> np.ndarray:
        """Finite-difference columns (all, or the listed ones) at x0."""
        base = self.apply(x0)
        idx = range(self.n) if cols is None else cols
        out = np.empty((self.n, len(idx)))
        for c, j in enumerate(idx):
            x = x0.copy()
            x[j] += eps
            out[:, c] = (self.apply(x) - base) / eps
        return out

    def spectral_radius(self, x0: np.ndarray, eps: float = 1e-7, dense_max: int = 2000, k: int = 1,
                        tol: float = 1e-6, ncv: int = 24, maxiter: int = 2000, stiff: bool = False) -> float:
        """Largest |eigenvalue| of the finite-difference step map at x0:
        dense below dense_max unknowns, else Arnoldi (k eigenvalues of
        largest modulus, Krylov space ncv, relative tolerance tol).

        stiff=True runs Arnoldi on G - I instead and returns the largest
        |mu + 1| over its k eigenvalues mu of largest modulus: for a stable
        base state the eigenvalues of G cluster at 1 - O(H), where Arnoldi on
        G converges slowly, while the modes that leave the unit disc first as
        H grows are the stiff ones, far from 1 and quick to converge on G - I.
        (A slow mode just outside the disc would be missed.)"""
        if self.n <= dense_max:
            G = self.columns(x0, eps)
            return float(np.max(np.abs(np.linalg.eigvals(G))))
        from scipy.sparse.linalg import LinearOperator, eigs
        base = self.apply(x0)
        scale = max(np.max(np.abs(x0)), 1.0)

        shift = 1.0 if stiff else 0.0

        def mv(v):
            v = np.asarray(v, dtype=float).ravel()
            nrm = np.linalg.norm(v)
            if nrm == 0.0:
                return np.zeros_like(v)
            e = eps * scale / nrm
            return (self.apply(x0 + e * v) - base) / e - shift * v

        op = LinearOperator((self.n, self.n), matvec=mv, dtype=float)
        vals = eigs(op, k=k, which="LM", tol=tol, ncv=ncv, maxiter=maxiter, return_eigenvectors=False)
        return float(np.max(np.abs(vals + shift)))


def largest_stable_macrostep(make: Callable[[], System], H_lo: float, H_hi: float, step_tol: float = 1e-4,
                             eps: float = 1e-7, warm: int = 0, margin: float = 1e-9,
                             log: Optional[Callable[[str], None]] = None, **kw) -> float:
    """Largest macrostep H in [H_lo, H_hi] (to step_tol) at which the step matrix
    about the system's started state has spectral radius at most 1 + margin
    (the margin covers the finite-difference and Arnoldi error).  make()
    returns a fresh System; each trial sets H, bootstraps, takes `warm`
    macrosteps and linearises one macrostep there; kw go to
    StepMap.spectral_radius."""
    def stable(H):
        s = make()
        s.set_macrostep(H)
        s.start(0.0)
        if warm:
            s.macrostep(warm)
        sm = StepMap(s)
        x0 = sm.pack()
        rho = sm.spectral_radius(x0, eps=eps, **kw)
        s.close()
        if log:
            log(f"H={H:.6g} rho={rho:.8f}")
        return rho <= 1.0 + margin

    lo, hi = H_lo, H_hi
    if not stable(lo):
        raise ValueError("lower end is not stable")
    if stable(hi):
        return hi
    while hi - lo > step_tol:
        mid = 0.5 * (lo + hi)
        if stable(mid):
            lo = mid
        else:
            hi = mid
    return lo


def perturbation_growth(sysg: System, nsteps: int = 500, amp: float = 1e-8, seed: int = 0) -> float:
    """Growth of a seeded random perturbation (relative size amp) of the
    started system's states over nsteps macrosteps: |y_N - y_N^0| / |dy_0|
    against an unperturbed copy run alongside.  For a steady base state this
    is power iteration on the step map: it exceeds any fixed bound once an
    eigenvalue leaves the unit disc, quickly when it leaves clearly."""
    x = [sysg.state(g) for g in range(sysg.ngrids)]
    hist = [[sysg.history(g, j) for j in range(sysg.wl.params["hist_len"])] for g in range(sysg.ngrids)]
    gen = torch.Generator(device="cpu").manual_seed(seed)
    dx = [amp * torch.randn(t.shape, generator=gen, dtype=torch.float64).to(t.device) * t.abs().max()
          for t in x]
    n0 = torch.sqrt(sum((d * d).sum() for d in dx)).item()
    ref = []
    for pert in (False, True):
        for g in range(sysg.ngrids):
            for j, h in enumerate(hist[g]):
                sysg.set_history(g, j, h)
        sysg.set_states([x[g] + dx[g] if pert else x[g] for g in range(sysg.ngrids)])
        sysg.resume(0.0)
        sysg.macrostep(nsteps)
        y = [sysg.state(g) for g in range(sysg.ngrids)]
        if not pert:
            ref = y
    d = torch.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(y, ref))).item()
    return d / n0 if np.isfinite(d) else float("inf")


def largest_stable_by_growth(make: Callable[[], System], H_lo: float, H_hi: float, step_tol: float,
                             nsteps: int = 500, bound: float = 100.0,
                             log: Optional[Callable[[str], None]] = None) -> float:
    """Largest macrostep H in [H_lo, H_hi] (to step_tol) whose perturbation
    growth over nsteps macrosteps stays below bound."""
    def stable(H):
        s = make()
        s.set_macrostep(H)
        s.start(0.0)
        gr = perturbation_growth(s, nsteps)
        s.close()
        if log:
            log(f"H={H:.6g} growth={gr:.4g}")
        return gr < bound

    lo, hi = H_lo, H_hi
    if not stable(lo):
        raise ValueError("lower end is not stable")
    if stable(hi):
        return hi
    while hi - lo > step_tol:
        mid = 0.5 * (lo + hi)
        if stable(mid):
            lo = mid
        else:
            hi = mid
    return lo

