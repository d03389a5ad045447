"""Stability tooling of the oracle (test infrastructure only).

Paper passages:
  * section "Extended-History Adams-Bashforth Schemes": the step matrix G of
    an AB scheme applied to dy/dt = -beta y, acting on (y_n, y_{n-1}, ...),
    and the eigenvalues of G^T G for the third-order case;
  * section "Procedure for Determining Discrete Stability": step matrices
    formed column by column by finite differences of one integrator step
    (perturbation 1e-7 of one entry of the integrator state, which for AB
    includes the right-hand-side history), stable when the spectral radius is
    at most 1; the largest stable step is searched to 1e-4;
  * section "Validation of the approximate stability calculation via RK4":
    RK4 on 1D advection, 61 points on a periodic domain of length 1.01666;
  * Appendix "Plotting Approximate Stability Regions": march dy/dt = k y with
    unit step for 100 steps along rays k = c + r e^{i theta}; a run is
    unstable once |y| exceeds 2; bisection on r.

Reading (listed in the design notes): the appendix prints the ray origin as
"+ 0.3"; with that origin y' = 0.3 y itself grows past 2 within 100 steps, so
the marching test fails at r = 0 for every integrator.  The rays here start
from a point c inside the region (default -0.1, inside the regions of every
scheme used here), which is the boundary-locus construction the appendix names.
"""
from fractions import Fraction as Fr
from typing import Callable, List, Sequence

import numpy as np

from .coeffs import ab_coefficients
from .sbp import dense_D


# --------------------------------------------------------------- scalar ODE
def ab_alpha(order: int, hist_len: int) -> List[float]:
    """AB coefficients for unit step, oldest first."""
    return [float(a) for a in ab_coefficients(order, hist_len, Fr(1))]


def ab_scalar_G(alpha_oldest_first: Sequence[float], beta: float) -> np.ndarray:
    """The step matrix of the AB scheme on dy/dt = -beta y acting on
    (y_n, y_{n-1}, ..., y_{n-m+1}): first row 1 - beta a_1, -beta a_2, ...
    with a_1 the weight of the newest value; a shift below."""
    a = list(reversed(list(alpha_oldest_first)))     # newest first
    m = len(a)
    G = np.zeros((m, m))
    G[0, :] = [-beta * x for x in a]
    G[0, 0] += 1.0
    for i in range(1, m):
        G[i, i - 1] = 1.0
    return G


def ab34_gtg_eigs_paper(alpha_oldest_first: Sequence[float], beta: float) -> np.ndarray:
    """Eigenvalues of G^T G for a three-value history as the paper states
    them: 1 and (C +- sqrt(C^2 - 4 a_3^2 beta^2)) / 2 with
    C = -2 a_1 beta + 2 + beta^2 |a|^2."""
    a = list(reversed(list(alpha_oldest_first)))
    C = -2.0 * a[0] * beta + 2.0 + beta * beta * sum(x * x for x in a)
    disc = np.sqrt(complex(C * C - 4.0 * a[2] ** 2 * beta ** 2))
    return np.array([1.0, (C + disc).real / 2.0, (C - disc).real / 2.0])


def march_ab(alpha_oldest_first: Sequence[float], k: complex, nsteps: int = 100, bound: float = 2.0) -> bool:
    """True when AB with unit step keeps |y| <= bound for nsteps steps of
    dy/dt = k y from the exact history y(t_j) = exp(k t_j), t_j = -(m-1)..0."""
    a = list(alpha_oldest_first)
    m = len(a)
    ys = [np.exp(k * j) for j in range(-(m - 1), 1)]
    F = [k * y for y in ys]
    y = ys[-1]
    for _ in range(nsteps):
        y = y + sum(a[j] * F[j] for j in range(m))
        if not abs(y) <= bound:
            return False
        F = F[1:] + [k * y]
    return True


def rk4_amplification(z: complex) -> complex:
    return 1.0 + z + z * z / 2.0 + z ** 3 / 6.0 + z ** 4 / 24.0


def march_rk4(k: complex, nsteps: int = 100, bound: float = 2.0) -> bool:
    y = 1.0 + 0.0j
    R = rk4_amplification(k)
    for _ in range(nsteps):
        y = R * y
        if not abs(y) <= bound:
            return False
    return True


def ray_boundary(stable: Callable[[complex], bool], theta: float, centre: complex = -0.1,
                 rmax: float = 8.0, tol: float = 1e-9) -> float:
    """Largest r (to tol) with stable(centre + r e^{i theta}), by bisection
    from r = 0 (assumed stable) and r = rmax (assumed unstable)."""
    d = np.exp(1j * theta)
    lo, hi = 0.0, rmax
    if stable(centre + hi * d):
        return hi
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if stable(centre + mid * d):
            lo = mid
        else:
            hi = mid
    return lo


def ab_root_stable(alpha_oldest_first: Sequence[float], z: complex) -> bool:
    """Root condition of the AB characteristic polynomial
    zeta^m - zeta^(m-1) - z sum_j a_j zeta^j (j = 0 oldest)."""
    a = list(alpha_oldest_first)
    m = len(a)
    p = np.zeros(m + 1, dtype=complex)
    p[0], p[1] = 1.0, -1.0
    for j, x in enumerate(a):
        p[m - j] -= z * x
    return float(np.max(np.abs(np.roots(p)))) <= 1.0 + 1e-12


# ------------------------------------------------------------ step matrices
def step_matrix(step: Callable[[np.ndarray], np.ndarray], x0: np.ndarray, eps: float = 1e-7) -> np.ndarray:
    """Columns (step(x0 + eps e_j) - step(x0)) / eps."""
    base = step(x0)
    n = x0.size
    G = np.empty((base.size, n))
    for j in range(n):
        x = x0.copy()
        x[j] += eps
        G[:, j] = (step(x) - base) / eps
    return G


def spectral_radius(G: np.ndarray) -> float:
    return float(np.max(np.abs(np.linalg.eigvals(G))))


def largest_stable(stable: Callable[[float], bool], lo: float, hi: float, tol: float = 1e-4) -> float:
    """Largest dt in [lo, hi] with stable(dt), to tol, by bisection (lo
    stable, hi unstable)."""
    if not stable(lo):
        raise ValueError("lower end is not stable")
    if stable(hi):
        return hi
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if stable(mid):
            lo = mid
        else:
            hi = mid
    return lo


def rk4_advection_dt_max(n: int = 61, length: float = 1.01666, sbp: int = 42, tol: float = 1e-5) -> float:
    """RK4 on u_t + u_x = 0, periodic, n points spaced length / n, the
    interior SBP stencil; largest dt with spectral radius of the
    finite-difference step matrix at most 1 (+1e-9 for the rounding of the
    columns)."""
    dx = length / n
    D = np.array(dense_D(sbp, n, periodic=True), dtype=float) / dx

    def rhs(u):
        return -(D @ u)

    def stable(dt):
        def step(u):
            k1 = rhs(u)
            k2 = rhs(u + 0.5 * dt * k1)
            k3 = rhs(u + 0.5 * dt * k2)
            k4 = rhs(u + dt * k3)
            return u + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        G = step_matrix(step, np.zeros(n), eps=1e-7)
        return spectral_radius(G) <= 1.0 + 1e-9

    return largest_stable(stable, 0.01, 0.05, tol)


# ----------------------------------------------------- MRAB step matrices
def mrab_state(mr) -> np.ndarray:
    """Integrator state of an oracle MRAB object: every grid's state, then
    its history values oldest first."""
    parts = []
    for g in range(len(mr.y)):
        parts.append(mr.y[g].ravel())
        parts.extend(h.ravel() for h in mr.hist[g])
    return np.concatenate(parts)


def mrab_step(mr, x: np.ndarray) -> np.ndarray:
    """One macrostep of the oracle MRAB object from integrator state x."""
    shapes = [a.shape for a in mr.y]
    m = mr.m
    y, hist, off = [], [], 0
    for g, sh in enumerate(shapes):
        n = int(np.prod(sh))
        y.append(x[off:off + n].reshape(sh).copy())
        off += n
        hs = []
        for _ in range(m):
            hs.append(x[off:off + n].reshape(sh).copy())
            off += n
        hist.append(hs)
    t = mr.t
    mr.set_history(y, hist, t)
    mr.macrostep()
    out = mrab_state(mr)
    mr.set_history(y, hist, t)
    return out


def mrab_spectral_radius(mr, x0: np.ndarray, eps: float = 1e-7, k: int = 1, tol: float = 1e-6,
                         ncv: int = 24, maxiter: int = 2000, stiff: bool = False) -> float:
    """Spectral radius of the finite-difference step map of one oracle MRAB
    macrostep about x0: Arnoldi (scipy) on v -> (step(x0 + e v) - step(x0)) / e
    with e = eps * max(1, |x0|_inf) / |v|; dense columns below 2000
    unknowns."""
    step = lambda x: mrab_step(mr, x)  # noqa: E731
    if x0.size < 2000:
        return spectral_radius(step_matrix(step, x0, eps))
    from scipy.sparse.linalg import LinearOperator, eigs
    base = step(x0)
    scale = max(float(np.max(np.abs(x0))), 1.0)

    shift = 1.0 if stiff else 0.0    # stiff: Arnoldi on G - I, largest |mu + 1|

    def mv(v):
        v = np.asarray(v, dtype=float).ravel()
        nrm = np.linalg.norm(v)
        if nrm == 0.0:
            return np.zeros_like(v)
        e = eps * scale / nrm
        return (step(x0 + e * v) - base) / e - shift * v

    op = LinearOperator((x0.size, x0.size), matvec=mv, dtype=float)
    vals = eigs(op, k=k, which="LM", tol=tol, ncv=ncv, maxiter=maxiter, return_eigenvectors=False)
    return float(np.max(np.abs(vals + shift)))
