"""Diagonal-norm SBP first-derivative operators, in exact rationals.

Part of the test oracle (test infrastructure only).

Paper: section "The Compressible Navier-Stokes Equations on Overset Meshes"
names the SBP operators of Strand / Mattsson-Nordstrom and uses the
third-order (interior order 4, boundary order 2) diagonal-norm operator; the
Appendix "Spatial Accuracy of Right-Hand Sides" states the resulting orders
(p at the boundary, 2p inside).  The coefficients themselves are not printed in
the paper; the tables below are the classical diagonal-norm families, accepted
only because the exact summation-by-parts identity H D + D^T H = B and the
accuracy conditions hold (see tests/test_oracle_sbp.py).

Index-space spacing is 1.  Right-end rows mirror the left-end rows with
negated signs: D[N-1-i, N-1-j] = -D[i, j].
"""
from fractions import Fraction as Fr

SBP21 = dict(
    name="SBP 2-1",
    interior={-1: Fr(-1, 2), 1: Fr(1, 2)},
    closure=[[Fr(-1), Fr(1)]],
    norm=[Fr(1, 2)],
    half_width=1,
)

SBP42 = dict(
    name="SBP 4-2",
    interior={-2: Fr(1, 12), -1: Fr(-2, 3), 1: Fr(2, 3), 2: Fr(-1, 12)},
    closure=[
        [Fr(-24, 17), Fr(59, 34), Fr(-4, 17), Fr(-3, 34), Fr(0), Fr(0)],
        [Fr(-1, 2), Fr(0), Fr(1, 2), Fr(0), Fr(0), Fr(0)],
        [Fr(4, 43), Fr(-59, 86), Fr(0), Fr(59, 86), Fr(-4, 43), Fr(0)],
        [Fr(3, 98), Fr(0), Fr(-59, 98), Fr(0), Fr(32, 49), Fr(-4, 49)],
    ],
    norm=[Fr(17, 48), Fr(59, 48), Fr(43, 48), Fr(49, 48)],
    half_width=2,
)

TABLES = {21: SBP21, 42: SBP42}


def table(sbp: int) -> dict:
    return TABLES[sbp]


def nclosure(sbp: int) -> int:
    return len(TABLES[sbp]["closure"])


def closure_width(sbp: int) -> int:
    return len(TABLES[sbp]["closure"][0])


def p0(sbp: int) -> Fr:
    """(1,1) entry of the norm matrix H (index spacing 1)."""
    return TABLES[sbp]["norm"][0]


def dense_D(sbp: int, n: int, periodic: bool = False):
    """Full-line first-derivative matrix (list of lists of Fractions)."""
    t = TABLES[sbp]
    D = [[Fr(0)] * n for _ in range(n)]
    if periodic:
        for i in range(n):
            for off, c in t["interior"].items():
                D[i][(i + off) % n] += c
        return D
    nb = len(t["closure"])
    if n < 2 * nb:
        raise ValueError("line shorter than two closures")
    for i in range(nb):
        for j, c in enumerate(t["closure"][i]):
            D[i][j] = c
            D[n - 1 - i][n - 1 - j] = -c
    for i in range(nb, n - nb):
        for off, c in t["interior"].items():
            D[i][i + off] = c
    return D


def dense_H(sbp: int, n: int, periodic: bool = False):
    if periodic:
        return [Fr(1)] * n
    t = TABLES[sbp]
    nb = len(t["norm"])
    h = [Fr(1)] * n
    for i in range(nb):
        h[i] = t["norm"][i]
        h[n - 1 - i] = t["norm"][i]
    return h


def as_float_arrays(sbp: int):
    """(interior[5] for offsets -2..2, closure rows padded to 4x6, nclosure, p0)."""
    t = TABLES[sbp]
    interior = [float(t["interior"].get(o, Fr(0))) for o in (-2, -1, 0, 1, 2)]
    clo = [[0.0] * 6 for _ in range(4)]
    for i, row in enumerate(t["closure"]):
        for j, c in enumerate(row):
            clo[i][j] = float(c)
    return interior, clo, len(t["closure"]), float(t["norm"][0])
