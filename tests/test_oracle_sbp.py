"""Pins of the oracle's SBP operators and of its run-based derivative.

The SBP tables are checked against the definition of a diagonal-norm
summation-by-parts operator (H D + D^T H = diag(-1, 0, ..., 0, 1), exactly, in
rationals) and against the accuracy orders the paper states (boundary order
p, interior order 2p: Appendix "Spatial Accuracy of Right-Hand Sides"), and the
periodic fourth-order spectrum against the value the paper prints (Lele's
lambda_max dx = 1.3722).
"""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import sbp

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.mark.parametrize("k", [21, 42])
@pytest.mark.parametrize("n", [8, 9, 12, 17])
def test_sbp_property_exact(k, n):
    D = sbp.dense_D(k, n)
    H = sbp.dense_H(k, n)
    for i in range(n):
        for j in range(n):
            v = H[i] * D[i][j] + H[j] * D[j][i]
            want = Fr(-1) if i == j == 0 else (Fr(1) if i == j == n - 1 else Fr(0))
            assert v == want, (i, j, v)


@pytest.mark.parametrize("k,bdry,inner", [(21, 1, 2), (42, 2, 4)])
def test_sbp_accuracy_orders(k, bdry, inner):
    n = 16
    D = sbp.dense_D(k, n)
    nb = sbp.nclosure(k)
    for deg in range(inner + 2):
        f = [Fr(i) ** deg for i in range(n)]
        df = [deg * Fr(i) ** (deg - 1) if deg else Fr(0) for i in range(n)]
        res = [sum(D[i][j] * f[j] for j in range(n)) - df[i] for i in range(n)]
        for i in range(n):
            closure = i < nb or i >= n - nb
            exact_expected = deg <= (bdry if closure else inner)
            if exact_expected:
                assert res[i] == 0, (k, deg, i)
        # the interior order is not higher than claimed
        if deg == inner + 1:
            assert any(res[i] != 0 for i in range(nb, n - nb))


def test_periodic_42_spectrum_matches_paper():
    n = 480
    D = np.array([[float(c) for c in row] for row in sbp.dense_D(42, n, periodic=True)])
    lam = np.linalg.eigvals(D)
    assert np.max(np.abs(lam.real)) < 1e-12
    assert abs(np.max(np.abs(lam.imag)) - GOLD["lele_periodic_4th_order_max_lambda_dx"]["value"]) < 5e-4
    # RK4 dt estimate printed in the same passage
    g = GOLD["rk4_advection_dt_max"]
    est = GOLD["rk4_imag_axis_bound"]["value"] / np.max(np.abs(lam.imag)) * g["dx"]
    assert abs(est - g["value"]) < 2e-4


@pytest.mark.parametrize("k", [21, 42])
def test_oracle_run_derivative_matches_dense(k):
    """orc_deriv (runs with holes, periodic wrap) equals the dense per-run
    operator applied line by line."""
    import workloads
    from oracle import OracleSystem
    wl = workloads.mms_box(48, viscous=False, sbp=k)
    s = OracleSystem(wl)
    rng = np.random.default_rng(0)
    for g in range(2):
        grid = wl.grids[g]
        f = rng.standard_normal(grid.npts)
        for d in range(2):
            out = s.deriv(g, f, d)
            pos, rlen, _, _ = s.grids[g].run_info[d]
            nx, ny = grid.n
            F = f.reshape(ny, nx)
            O = out.reshape(ny, nx)
            lines = range(ny) if d == 0 else range(nx)
            for li in lines:
                line = F[li, :] if d == 0 else F[:, li]
                oline = O[li, :] if d == 0 else O[:, li]
                idx = [li * nx + i for i in range(nx)] if d == 0 else [j * nx + li for j in range(ny)]
                L = len(line)
                # group points by run start
                seen = set()
                for t, p in enumerate(idx):
                    if rlen[p] < 0 or p in seen:
                        continue
                    if rlen[p] == 0:
                        Dm = np.array([[float(c) for c in r] for r in sbp.dense_D(k, L, periodic=True)])
                        np.testing.assert_allclose(oline, Dm @ line, atol=1e-12)
                        seen.update(idx)
                        continue
                    start = (t - pos[p]) % L
                    run = [(start + r) % L for r in range(rlen[p])]
                    Dm = np.array([[float(c) for c in r] for r in sbp.dense_D(k, rlen[p])])
                    np.testing.assert_allclose(oline[run], Dm @ line[run], atol=1e-12)
                    seen.update(idx[r] for r in run)
