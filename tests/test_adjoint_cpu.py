"""Discrete-adjoint support that runs without a GPU: the oracle's
objective and finite-difference helpers pinned to closed forms, and the
library's checkpointing schedule against the published optimum of binomial
checkpointing."""
from math import comb

import numpy as np
import pytest

import workloads
from oracle import OracleSystem
from oracle.adjoint import pressure, richardson, run_objective


def test_richardson_exact_for_quartics():
    """One Richardson step on central differences cancels the h^2 term:
    exact (to rounding) for polynomials up to degree 4."""
    f = lambda e: 3.0 + 2.0 * e + 5.0 * e ** 2 - 7.0 * e ** 3 + 11.0 * e ** 4  # noqa: E731
    assert abs(richardson(f, 0.1) - 2.0) < 1e-13
    g = lambda e: e ** 5  # noqa: E731
    assert abs(richardson(g, 0.1) - 0.0) > 1e-6     # degree 5 is not


def test_pressure_closed_form():
    gamma = 1.4
    rho, u, v, p = 1.3, 0.7, -0.2, 2.5
    q = np.array([[rho], [rho * u], [rho * v], [p / (gamma - 1) + 0.5 * rho * (u * u + v * v)]])
    assert abs(pressure(q, gamma)[0] - p) < 1e-14


def test_objective_of_a_steady_state():
    """Uniform flow is a steady state of the cylinder case without a wall:
    the trapezoid rule over the objective grid's own-step times then gives
    J = (nmacro H) p_inf sum_k w_k."""
    wl = workloads.cylinder(nbg=64, ntheta=48, nr=24, half=5.0, wall=False, perturb=0.0)
    orc = OracleSystem(wl)
    h, H = orc.timestep()
    y0 = [np.asarray(q, dtype=np.float64).reshape(4, -1) for q in wl.q0]
    pts = np.arange(0, 48 * 24, 7)
    w = np.linspace(0.5, 1.5, len(pts))
    nmacro = 2
    J, _ = run_objective(orc, y0, nmacro, H, 1, pts, w)
    p_inf = pressure(y0[1][:, :1], wl.params["gamma"])[0]
    want = nmacro * H * p_inf * float(np.sum(w))
    assert abs(J - want) <= 1e-9 * want


def test_schedule_matches_binomial_optimum():
    """Reversing l steps with s snapshot slots (one holding the start): the
    forward steps a schedule recomputes, beyond the l recorded ones, are at
    least t l - C(s + t, t - 1) for the t with C(s + t - 1, t - 1) < l <=
    C(s + t, t), and the binomial schedule attains it."""
    from paper_1805_06607_amd.adjoint import schedule_cost
    for s in range(1, 7):
        for l in range(1, 60):
            t = 0
            while comb(s + t, t) < l:
                t += 1
            opt = t * l - comb(s + t, t - 1) if t > 0 else 0
            assert schedule_cost(l, s) - l == opt, (l, s)
    assert schedule_cost(200, 20) - 200 == 2 * 200 - comb(22, 1)


def test_schedule_rejects_bad_arguments():
    from paper_1805_06607_amd import _lib
    from paper_1805_06607_amd.adjoint import schedule_cost
    with pytest.raises(_lib.MrabError):
        schedule_cost(10, 0)
    with pytest.raises(_lib.MrabError):
        schedule_cost(5000, 3)
