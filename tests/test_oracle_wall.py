"""The oracle's isothermal no-slip wall penalty enforces the wall condition
weakly: the slip velocity and the wall temperature error at the wall points
go to zero under grid refinement (section "Guiding Experiment" uses an
isothermal no-slip wall; its penalty form comes from a reference the paper
does not reproduce).

Channel periodic in x between two walls, started impulsively at u = 1 with the
walls 5 % hotter than the gas, advanced to t = 0.1 with classic RK4 on the
oracle's right-hand side at 33, 65 and 129 points across.  Without the viscous
part of the penalty the slip stays at 1 (the inviscid part leaves the
tangential velocity free at a wall), which this test would catch."""
import math

import numpy as np
import pytest

import workloads
from oracle import OracleSystem
from oracle.integrate import rk4_steps


def wall_residuals(ny, T=0.1):
    wl = workloads.wall_channel(ny)
    orc = OracleSystem(wl)
    _, H = orc.timestep()
    n = int(math.ceil(T / (2.0 * H)))
    y = rk4_steps(orc.rhs, wl.q0, T / n, n)[0]
    nx, nyy = wl.grids[0].n
    gm1 = wl.params["gamma"] - 1.0
    rho = y[0].reshape(nyy, nx)
    u = y[1].reshape(nyy, nx) / rho
    v = y[2].reshape(nyy, nx) / rho
    p = gm1 * (y[3].reshape(nyy, nx) - 0.5 * rho * (u * u + v * v))
    Tw = wl.params["T_wall"]
    walls = [0, nyy - 1]
    slip = max(float(np.max(np.abs(u[j]))) for j in walls)
    terr = max(float(np.max(np.abs(p[j] / rho[j] - Tw))) / Tw for j in walls)
    core = float(np.max(np.abs(u[nyy // 2] - 1.0)))
    return slip, terr, core


def test_wall_slip_and_temperature_error_vanish_under_refinement():
    res = [wall_residuals(ny) for ny in (33, 65, 129)]
    slips = [r[0] for r in res]
    terrs = [r[1] for r in res]
    for a, b in zip(slips, slips[1:]):
        assert b < a / 4.0, slips
    for a, b in zip(terrs, terrs[1:]):
        assert b < a / 4.0, terrs
    assert slips[-1] < 1e-3 and terrs[-1] < 1e-4, (slips, terrs)
    # the core flow, outside the boundary layers, is still the initial stream
    assert all(r[2] < 1e-6 for r in res), res
