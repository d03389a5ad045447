"""Pins of the oracle's overset assembly (section "SAT-Based Interpolation"):
hole counts and receivers on the vortex box-in-box case, donor choice against a
brute-force search, Lagrange interpolation reproducing polynomials of degree
< width per direction, and rejection of runs shorter than two closures.
"""
import itertools
import math

import numpy as np
import pytest

import workloads
from oracle import OracleSystem, overset


def test_vortex_box_hole_and_receivers():
    wl = workloads.vortex_box()
    s = OracleSystem(wl)
    ib0 = s.grids[0].iblank
    assert int((ib0 == 0).sum()) == 121          # 11 x 11 blanked points
    assert len(s.grids[0].recv_pts) == 44        # hole rim, corners excluded
    assert len(s.grids[1].recv_pts) == 4 * 32 - 4
    X = wl.grids[0].points()
    holes = np.nonzero(ib0 == 0)[0]
    assert np.all(np.maximum(np.abs(X[0, holes] - 5), np.abs(X[1, holes] - 5)) < 11.5 * 10 / 128)


def _brute_force_donor(grids, iblanks, g, x, width):
    """Enumerate every cell of every other grid; keep the valid W-stencils
    whose central cell contains x; pick by (priority desc, grid id, base)."""
    best = None
    for dg, grid in enumerate(grids):
        if dg == g or grid.kind != workloads.CARTESIAN:
            continue
        dim = grid.dim
        for base in itertools.product(*[range(-width, grid.n[d]) for d in range(dim)]):
            ok = True
            idx = []
            for d in range(dim):
                lo = grid.origin[d] + (base[d] + width // 2 - 1) * grid.spacing[d]
                hi = lo + grid.spacing[d]
                if not (lo <= x[d] < hi):
                    ok = False
                    break
                ids = [base[d] + a for a in range(width)]
                if grid.periodic[d]:
                    ids = [i % grid.n[d] for i in ids]
                elif ids[0] < 0 or ids[-1] >= grid.n[d]:
                    ok = False
                    break
                idx.append(ids)
            if not ok:
                continue
            pts = []
            for a in itertools.product(*[range(width)] * dim):
                p = 0
                st = 1
                for d in range(dim):
                    p += idx[d][a[d]] * st
                    st *= grid.n[d]
                pts.append(p)
            if not all(iblanks[dg][p] for p in pts):
                continue
            key = (-grid.priority, dg)
            if best is None or key < best[0]:
                best = (key, dg, sorted(pts))
    return best


def test_donor_search_matches_brute_force():
    wl = workloads.vortex_box(nbg=24, npatch=16)
    s = OracleSystem(wl)
    iblanks = [gr.iblank for gr in s.grids]
    for g in range(2):
        X = wl.grids[g].points()
        for r, p in enumerate(s.grids[g].recv_pts):
            dg, pts, _ = s.donor_tables[g][r]
            bf = _brute_force_donor(wl.grids, iblanks, g, X[:, p], 2)
            assert bf is not None
            assert bf[1] == dg and bf[2] == sorted(pts)


@pytest.mark.parametrize("width", [2, 4])
def test_lagrange_weights_reproduce_polynomials(width):
    rng = np.random.default_rng(width)
    for _ in range(20):
        s = rng.uniform(width // 2 - 1, width // 2)
        w = overset.lagrange_weights_1d(s, width)
        for deg in range(width):
            assert abs(sum(w[a] * a ** deg for a in range(width)) - s ** deg) < 1e-12


@pytest.mark.parametrize("sbp,width", [(21, 2), (42, 4)])
def test_receiver_data_reproduces_polynomial_state(sbp, width):
    """q_hat of every receiver equals a tensor polynomial (degree < width per
    direction) sampled on the donor grid, evaluated at the receiver."""
    wl = workloads.mms_box(40, viscous=False, sbp=sbp)
    s = OracleSystem(wl)

    def poly(X):
        x, y = X
        deg = width - 1
        return 1.5 + 0.3 * x ** deg * y ** (deg - 1) - 0.2 * y ** deg + 0.1 * x * y

    states = []
    for g in wl.grids:
        X = g.points()
        q = np.stack([2.0 + 0.1 * poly(X), 0.0 * X[0], 0.0 * X[0], 5.0 + poly(X)])
        states.append(q)
    for g in range(2):
        rd = s.receiver_data(g, states)
        X = wl.grids[g].points()[:, s.grids[g].recv_pts]
        np.testing.assert_allclose(rd[:, 3], 5.0 + poly(X), rtol=0, atol=1e-12)


def test_short_runs_are_rejected():
    """A hole leaving a periodic run of 7 points: fine for SBP 2-1 (needs 2),
    rejected for SBP 4-2 (needs 8)."""
    wl = workloads.vortex_box(nbg=12, npatch=20)
    g = wl.grids[0]
    ib = overset.blank(g)
    info = overset.runs(g, ib, 21)
    assert info[0][1].max() == 7
    with pytest.raises(overset.AssemblyError):
        overset.runs(g, ib, 42)
