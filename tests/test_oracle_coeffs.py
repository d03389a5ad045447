"""Pins of the oracle's Adams-Bashforth coefficients (eq. vandermonde, ext_ab).

Textbook closed forms of AB2-AB4, exact integration of every polynomial of
degree < n for any target offset, the minimum-norm property of the extended
history schemes, and the paper's statement that AB34/AB45 reach further along
the negative real axis than AB3/AB4.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle.coeffs import ab_coefficients, nodes


def test_textbook_adams_bashforth():
    assert ab_coefficients(1, 1) == [Fr(1)]
    assert ab_coefficients(2, 2) == [Fr(-1, 2), Fr(3, 2)]
    assert ab_coefficients(3, 3) == [Fr(5, 12), Fr(-16, 12), Fr(23, 12)]
    assert ab_coefficients(4, 4) == [Fr(-9, 24), Fr(37, 24), Fr(-59, 24), Fr(55, 24)]


@pytest.mark.parametrize("n,m", [(2, 2), (3, 3), (4, 4), (3, 4), (3, 5), (4, 5), (4, 6)])
@pytest.mark.parametrize("tau", [Fr(1), Fr(1, 2), Fr(1, 4), Fr(3, 4), Fr(2, 3)])
def test_exact_on_polynomials(n, m, tau):
    a = ab_coefficients(n, m, tau)
    t = nodes(m)
    for deg in range(n):
        lhs = sum(a[j] * t[j] ** deg for j in range(m))
        assert lhs == tau ** (deg + 1) / (deg + 1)
    # and not exact one degree higher (order is exactly n) for the square case
    if m == n:
        lhs = sum(a[j] * t[j] ** n for j in range(m))
        assert lhs != tau ** (n + 1) / (n + 1)


@pytest.mark.parametrize("n,m", [(3, 4), (3, 5), (4, 5), (4, 6)])
def test_extended_history_is_minimum_norm(n, m):
    a = ab_coefficients(n, m)
    t = nodes(m)
    V = np.array([[float(tj) ** i for i in range(n)] for tj in t])
    # a lies in the range of V
    z, *_ = np.linalg.lstsq(V, np.array([float(x) for x in a]), rcond=None)
    np.testing.assert_allclose(V @ z, [float(x) for x in a], atol=1e-13)
    # any other solution (standard AB_n on the newest n nodes, zero elsewhere) is longer
    other = [Fr(0)] * (m - n) + ab_coefficients(n, n)
    assert sum(x * x for x in a) < sum(x * x for x in other)


def _real_axis_reach(coef):
    """Largest x>0 such that AB with coefficients coef is stable for z = -x
    (all roots of the characteristic polynomial inside the unit disc)."""
    m = len(coef)

    def stable(z):
        # zeta^m - zeta^(m-1) - z * sum_j a_j zeta^j  (j = 0 oldest)
        p = np.zeros(m + 1)
        p[0] = 1.0
        p[1] = -1.0
        for j, a in enumerate(coef):
            p[m - j] -= z * float(a)
        return np.max(np.abs(np.roots(p))) <= 1.0 + 1e-12

    x = 0.0
    while x < 5.0 and stable(-(x + 1e-3)):
        x += 1e-3
    return x


def test_extended_history_reaches_further_on_negative_axis():
    assert _real_axis_reach(ab_coefficients(3, 4)) > _real_axis_reach(ab_coefficients(3, 3)) * 1.1
    assert _real_axis_reach(ab_coefficients(4, 5)) > _real_axis_reach(ab_coefficients(4, 4)) * 1.1
