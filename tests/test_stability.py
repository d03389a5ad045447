"""Stability tooling: the oracle's step-matrix and stability-region
procedures pinned to the paper and to closed forms, and the library's
boundary loci checked against the oracle (CPU only)."""
import json
import os

import numpy as np
import pytest

from oracle import stability as st
from oracle.integrate import MRAB

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("beta", [0.05, 0.3, 0.5, 1.1])
def test_ab3_gtg_eigenvalues_match_paper(beta):
    """Section "Extended-History Adams-Bashforth Schemes": eigenvalues of
    G^T G for AB3 on dy/dt = -beta y are 1 and (C +- sqrt(C^2 -
    4 a_3^2 beta^2)) / 2."""
    a = st.ab_alpha(3, 3)
    G = st.ab_scalar_G(a, beta)
    got = np.sort(np.linalg.eigvalsh(G.T @ G))
    want = np.sort(st.ab34_gtg_eigs_paper(a, beta))
    assert np.allclose(got, want, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("order,m,beta", [(3, 3, 0.3), (3, 4, 0.6), (4, 4, 0.2), (4, 5, 0.4), (3, 3, 0.7)])
def test_fd_step_matrix_of_mrab_matches_scalar_G(order, m, beta):
    """The finite-difference step matrix of the oracle's integrator on
    dy/dt = -beta y (state: y and its m right-hand-side values) has the
    spectral radius of the paper's step matrix G on (y_n, y_{n-1}, ...)."""
    def rhs(states, which):
        return {g: -beta * states[g] for g in which}
    mr = MRAB(rhs, [1], order, m, 1.0)
    mr.set_history([np.array([1.0])], [[np.array([-beta])] * m], 0.0)
    x0 = st.mrab_state(mr)
    G = st.step_matrix(lambda x: st.mrab_step(mr, x), x0, eps=1e-7)
    rho_fd = st.spectral_radius(G)
    rho_paper = st.spectral_radius(st.ab_scalar_G(st.ab_alpha(order, m), beta))
    assert abs(rho_fd - rho_paper) < 1e-6 * max(1.0, rho_paper)


def test_rk4_advection_dt_max():
    """Section "Validation of the approximate stability calculation via RK4":
    61 points, periodic, dx = 0.01666; the step-matrix search lands between
    0.03 and 0.035, at the closed form 2 sqrt(2) dx / max|symbol| (the
    paper's estimate 0.03377 uses its rounded bounds 2.78 and 1.3722)."""
    g = GOLD["rk4_advection_dt_max"]
    dt = st.rk4_advection_dt_max(61, 1.01666, tol=1e-6)
    assert 0.030 < dt < 0.035
    n = 61
    dx = 1.01666 / n
    th = 2 * np.pi * np.arange(n) / n
    sym = np.max(np.abs(4 / 3 * np.sin(th) - np.sin(2 * th) / 6))
    assert abs(dt - 2 * np.sqrt(2) * dx / sym) < 2e-6
    assert abs(dt - g["value"]) / g["value"] < 0.025


def test_rk4_imaginary_bound_by_marching():
    """Appendix procedure on the imaginary axis: the RK4 boundary sits just
    above the exact crossing 2 sqrt(2) (growth past 2 within 100 steps needs
    |R| > 2^(1/100)); the paper quotes about 2.78."""
    r = st.ray_boundary(st.march_rk4, np.pi / 2, centre=0.0)
    assert 2 * np.sqrt(2) <= r < 2 * np.sqrt(2) * 1.01
    assert abs(GOLD["rk4_imag_axis_bound"]["value"] - r) / r < 0.02


@pytest.mark.parametrize("order,m", [(3, 3), (3, 4), (4, 4), (4, 5)])
def test_marching_boundary_vs_root_condition(order, m):
    """The marching heuristic only flags growth it sees within 100 steps, so
    for the schemes of the paper's results (AB3, AB34, AB4, AB45) its boundary
    lies on or outside the root-condition boundary, close to it.  (With still
    longer histories, AB35 and AB46, transient growth past 2 pulls the
    marching boundary inside the root-condition one on the negative real
    axis.)"""
    a = st.ab_alpha(order, m)
    for th in (np.pi, 0.8 * np.pi, 0.65 * np.pi):
        r_root = st.ray_boundary(lambda z: st.ab_root_stable(a, z), th, tol=1e-8)
        r_march = st.ray_boundary(lambda z: st.march_ab(a, z), th, tol=1e-8)
        assert r_root - 1e-6 <= r_march <= 1.3 * r_root + 0.02


def test_root_condition_real_axis_closed_forms():
    """AB3 is stable on [-6/11, 0], AB4 on [-3/10, 0]."""
    for (order, lim) in ((3, 6 / 11), (4, 3 / 10)):
        a = st.ab_alpha(order, order)
        r = st.ray_boundary(lambda z: st.ab_root_stable(a, z), np.pi, centre=-0.05, tol=1e-10)
        assert abs(r + 0.05 - lim) < 1e-8


def test_library_loci_against_oracle():
    """The library's closed-form boundary loci: the real-axis reach equals
    the oracle's root-condition bisection; extended history reaches further
    along the negative real axis (AB34 > AB3, AB45 > AB4, AB35 > AB34)."""
    from paper_1805_06607_amd.stability import ab_boundary_locus, imag_axis_reach, real_axis_reach, rk4_boundary
    reach = {}
    for (order, m) in ((3, 3), (3, 4), (3, 5), (4, 4), (4, 5)):
        reach[(order, m)] = real_axis_reach(ab_boundary_locus(order, m, 2000))
        a = st.ab_alpha(order, m)
        r = st.ray_boundary(lambda z: st.ab_root_stable(a, z), np.pi, centre=-0.05, tol=1e-10) + 0.05
        assert abs(reach[(order, m)] - r) < 2e-3 * r
    assert abs(reach[(3, 3)] - 6 / 11) < 1e-9
    assert abs(reach[(4, 4)] - 3 / 10) < 1e-9
    assert reach[(3, 4)] > 1.1 * reach[(3, 3)] and reach[(4, 5)] > 1.1 * reach[(4, 4)]
    assert reach[(3, 5)] > reach[(3, 4)]
    z = rk4_boundary(2000, normalise=False)
    assert abs(imag_axis_reach(z) - 2 * np.sqrt(2)) < 1e-3
    assert abs(real_axis_reach(z) - 2.785293563) < 1e-6
    assert abs(imag_axis_reach(rk4_boundary(2000)) - 2 * np.sqrt(2) / 4) < 1e-3
