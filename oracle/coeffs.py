"""Adams-Bashforth coefficients from the Vandermonde system, in exact rationals.

Part of the test oracle (test infrastructure only).

Paper: section "Adams-Bashforth Integration", eq. (vandermonde) and
eq. (ab_general); section "Extended-History Adams-Bashforth Schemes",
eq. (ext_ab) (minimum 2-norm coefficients for m > n history values).

Reading (the printed index range is ambiguous): history nodes are measured in
units of the level's own step, newest node at 0 and older nodes negative,
t_j = -(m-1-j) for j = 0..m-1 (oldest first).  For a target offset tau the
right-hand side is b_i = tau^(i+1)/(i+1), i = 0..n-1 (the integral of the
monomial t^i from 0 to tau) and V[j][i] = t_j^i.  For m = n, V^T alpha = b; for
m > n, alpha = V (V^T V)^(-1) b, the minimum-norm solution.  Coefficients are
exact rationals, rounded once to double by the caller, then scaled by the step.
"""
from fractions import Fraction as Fr
from typing import List


def _solve(A: List[List[Fr]], b: List[Fr]) -> List[Fr]:
    """Gaussian elimination with exact rationals (A square, nonsingular)."""
    n = len(A)
    M = [list(map(Fr, A[i])) + [Fr(b[i])] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [M[r][k] - f * M[c][k] for k in range(n + 1)]
    return [M[i][n] / M[i][i] for i in range(n)]


def nodes(hist_len: int) -> List[Fr]:
    return [Fr(-(hist_len - 1 - j)) for j in range(hist_len)]


def ab_coefficients(order: int, hist_len: int, tau=Fr(1)) -> List[Fr]:
    """alpha_j (oldest first) such that y(t0 + tau) ~ y(t0) + sum_j alpha_j F_j,
    in units where the history spacing is 1."""
    n, m = order, hist_len
    if m < n or n < 1:
        raise ValueError("need hist_len >= order >= 1")
    tau = Fr(tau)
    t = nodes(m)
    V = [[t[j] ** i for i in range(n)] for j in range(m)]
    b = [tau ** (i + 1) / (i + 1) for i in range(n)]
    if m == n:
        VT = [[V[j][i] for j in range(m)] for i in range(n)]
        return _solve(VT, b)
    VtV = [[sum(V[k][i] * V[k][j] for k in range(m)) for j in range(n)] for i in range(n)]
    z = _solve(VtV, b)
    return [sum(V[j][i] * z[i] for i in range(n)) for j in range(m)]


def ab_coefficients_float(order: int, hist_len: int, tau=Fr(1), step: float = 1.0) -> List[float]:
    return [float(a) * step for a in ab_coefficients(order, hist_len, tau)]
