"""Pins of the oracle's time integrators (section "Multi-rate Adams-Bashforth
Integration"): exact integration of polynomial right-hand sides, convergence
order n against the matrix exponential on a coupled fast/slow linear system,
and MRAB at step ratio 1 reproducing an independent single-rate AB loop bit for
bit.
"""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from oracle.coeffs import ab_coefficients
from oracle.integrate import MRAB, srab_steps


def poly_rhs(coefs_per_level):
    """Each level holds (y, tau) with tau' = 1 and y' = p_g(tau of level 0)."""
    def rhs(states, which):
        tau0 = states[0][1]
        out = {}
        for g in which:
            c = coefs_per_level[g]
            val = sum(ck * tau0 ** k for k, ck in enumerate(c))
            out[g] = np.array([val, 1.0])
        return out
    return rhs


@pytest.mark.parametrize("order,m", [(3, 3), (4, 4), (3, 4)])
@pytest.mark.parametrize("rates", [(1, 1), (1, 2), (1, 4), (1, 2, 4), (2, 3 * 2)])
def test_polynomial_exactness(order, m, rates):
    if any(max(rates) % r for r in rates):
        pytest.skip("rates must divide")
    # boot-strap RK integrates degree <= order-1 exactly: keep deg <= min(order-1, 2 or 3)
    deg = order - 1
    rng = np.random.default_rng(order * 10 + m)
    coefs = [list(rng.uniform(-1, 1, deg + 1)) for _ in rates]
    rhs = poly_rhs(coefs)
    H = 0.1
    mr = MRAB(rhs, list(rates), order, m, H)
    y0 = [np.array([0.0, 0.0]) for _ in rates]
    mr.bootstrap(y0, 0.0)
    for _ in range(7):
        mr.macrostep()
    t = mr.t
    for g, c in enumerate(coefs):
        exact = sum(ck * t ** (k + 1) / (k + 1) for k, ck in enumerate(c))
        assert abs(mr.y[g][0] - exact) < 1e-12 * max(1.0, abs(exact))
        assert abs(mr.y[g][1] - t) < 1e-13


def linear_system():
    # fast component (2x2 oscillator with damping) coupled weakly to a slow one
    A = np.array([[-0.5, 6.0, 0.3, 0.0],
                  [-6.0, -0.5, 0.0, 0.2],
                  [0.1, 0.0, -0.3, 0.5],
                  [0.0, -0.1, -0.5, -0.2]])
    blocks = [slice(0, 2), slice(2, 4)]

    def rhs(states, which):
        y = np.concatenate(states)
        f = A @ y
        return {g: f[blocks[g]] for g in which}
    return A, rhs


@pytest.mark.parametrize("order,m,sr", [(3, 3, 2), (3, 3, 4), (4, 4, 4), (3, 4, 3)])
def test_mrab_convergence_order(order, m, sr):
    A, rhs = linear_system()
    y0 = [np.array([1.0, 0.0]), np.array([0.5, -0.5])]
    T = 1.0
    errs = []
    for nsteps in (40, 80, 160):
        H = T / nsteps
        mr = MRAB(rhs, [1, sr], order, m, H)
        mr.bootstrap(y0, 0.0)
        t0 = mr.t
        nmac = nsteps - (m - 1)
        for _ in range(nmac):
            mr.macrostep()
        exact = expm(A * mr.t) @ np.concatenate(y0)
        errs.append(np.max(np.abs(np.concatenate(mr.y) - exact)))
    eoc = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert abs(eoc[-1] - order) < 0.35, (errs, eoc)


@pytest.mark.parametrize("order,m", [(3, 3), (4, 4), (3, 4)])
def test_mrab_ratio_one_is_srab_bitwise(order, m):
    A, rhs = linear_system()
    y0 = [np.array([1.0, 0.0]), np.array([0.5, -0.5])]
    H = 0.01
    mr = MRAB(rhs, [1, 1], order, m, H)
    mr.bootstrap(y0, 0.0)
    y, hist = [a.copy() for a in mr.y], [[h.copy() for h in hs] for hs in mr.hist]
    for _ in range(25):
        mr.macrostep()
    c = [float(a) * H for a in ab_coefficients(order, m)]
    ys, _ = srab_steps(rhs, y, hist, c, 25)
    for g in range(2):
        assert np.array_equal(mr.y[g], ys[g])
