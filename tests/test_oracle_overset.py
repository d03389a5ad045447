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


# ---------------------------------------------------------------- curvilinear donors
def test_omesh_mapping_samples_are_the_coordinates():
    """The O-mesh coordinates are the continuous mapping at integer indices."""
    g = workloads.cylinder(nbg=64, ntheta=96, nr=40, half=6.0).grids[1]
    I, J = np.meshgrid(np.arange(g.n[0]), np.arange(g.n[1]), indexing="xy")
    F = np.stack([I.ravel(), J.ravel()]).astype(float)
    assert np.array_equal(g.mapping(F), g.coords)


def test_omesh_inverse_returns_integer_indices_and_midpoints():
    """The closed-form inverse the product locates donors with returns the
    integer index at every O-mesh point and the fractional index at cell
    midpoints (theta modulo the period)."""
    g = workloads.cylinder().grids[1]
    nth = g.n[0]
    I, J = np.meshgrid(np.arange(g.n[0]), np.arange(g.n[1]), indexing="xy")
    for off in (0.0, 0.5):
        F = np.stack([I.ravel(), J.ravel()]).astype(float) + off
        F = F[:, F[1] <= g.n[1] - 1]
        got = g.inverse(g.mapping(F))
        di = np.mod(got[0] - F[0] + nth / 2, nth) - nth / 2
        assert np.max(np.abs(di)) < 1e-10
        assert np.max(np.abs(got[1] - F[1])) < 1e-10


def test_oracle_locate_inverts_the_mapping():
    """The oracle's own search (nearest point, then Newton) recovers random
    fractional indices, including next to the periodic seam."""
    g = workloads.cylinder(nbg=64, ntheta=96, nr=40, half=6.0).grids[1]
    rng = np.random.default_rng(5)
    F = np.stack([rng.uniform(0, g.n[0], 200), rng.uniform(0, g.n[1] - 1, 200)])
    F[0, :4] = [0.0, 1e-9, g.n[0] - 1e-9, 0.5]
    X = g.mapping(F)
    for k in range(F.shape[1]):
        f = overset.locate(g, X[:, k])
        di = (f[0] - F[0, k] + g.n[0] / 2) % g.n[0] - g.n[0] / 2
        assert abs(di) < 1e-9 and abs(f[1] - F[1, k]) < 1e-9, (k, f, F[:, k])


def _unwrapped_indices(grid, pts):
    """Index coordinates (dim, S) of a donor stencil's points, periodic
    directions unwrapped next to the first entry."""
    out = []
    rest = np.asarray(pts, dtype=np.int64)
    for d in range(grid.dim):
        i = (rest % grid.n[d]).astype(float)
        rest = rest // grid.n[d]
        if grid.periodic[d]:
            i = i[0] + (np.mod(i - i[0] + grid.n[d] / 2, grid.n[d]) - grid.n[d] / 2)
        out.append(i)
    return np.stack(out)


def test_curvilinear_donor_weights_reproduce_index_polynomials_and_location():
    """Cylinder: every background receiver's O-mesh stencil reproduces the
    index coordinates to degree 3 per direction (cubic Lagrange), and the
    mapping at the interpolated index is the receiver's own position."""
    wl = workloads.cylinder()
    s = OracleSystem(wl)
    om = wl.grids[1]
    X = wl.grids[0].points()
    n_checked = 0
    for r, p in enumerate(s.grids[0].recv_pts):
        dg, pts, wts = s.donor_tables[0][r]
        assert dg == 1
        F = _unwrapped_indices(om, pts)
        wts = np.asarray(wts)
        fhat = F @ wts
        for d in range(2):
            for k in range(4):
                assert abs(np.dot(wts, F[d] ** k) - fhat[d] ** k) < 1e-9 * max(1.0, abs(fhat[d]) ** k)
        xr = om.mapping(fhat[:, None])[:, 0]
        assert np.max(np.abs(xr - X[:, p])) < 1e-12
        n_checked += 1
    assert n_checked > 100


def _sparse(pts, wts):
    a = {}
    for q, w in zip(pts, wts):
        a[int(q)] = a.get(int(q), 0.0) + w
    return a


@pytest.mark.parametrize("case", ["cylinder_small", "cylinder", "vortex_box", "tgv3d_small", "vortex_convergence"])
def test_donor_tables_agree_with_product_assembly(case):
    """The oracle's donor search (its own location, loops) and the library's
    (mr_assemble_overset, host only: runs here without a device; curvilinear
    grids located by the problem's closed-form inverse) give the same
    blanking, the same receivers, the same donor grids and the same
    interpolation weights (as sparse vectors over donor points, so that a
    stencil base shifted at a node would still compare)."""
    from paper_1805_06607_amd.system import HostSetup
    wl = {"cylinder_small": lambda: workloads.cylinder(nbg=128, ntheta=96, nr=48),
          "cylinder": lambda: workloads.cylinder(),
          "vortex_box": lambda: workloads.vortex_box(),
          "tgv3d_small": lambda: workloads.tgv3d(nbg=48, npatch=24, ninner=16),
          "vortex_convergence": lambda: workloads.vortex_convergence(50)}[case]()
    s = OracleSystem(wl)
    h = HostSetup(wl)
    try:
        for g in range(len(wl.grids)):
            assert np.array_equal(s.grids[g].iblank, h.iblanks[g])
            assert np.array_equal(s.grids[g].recv_pts, h.recv_pts[g])
            pmap = {}
            for dg, (rr, pp, ww) in h.donor_tables[g].items():
                for k in range(len(rr)):
                    pmap[int(rr[k])] = (dg, pp[k], ww[k])
            assert len(pmap) == len(s.grids[g].recv_pts)
            for r, p in enumerate(s.grids[g].recv_pts):
                dg, pts, wts = s.donor_tables[g][r]
                pdg, ppts, pw = pmap[int(p)]
                assert dg == pdg
                a, b = _sparse(pts, wts), _sparse(ppts, pw)
                for k in set(a) | set(b):
                    assert abs(a.get(k, 0.0) - b.get(k, 0.0)) < 1e-12, (g, p, k)
    finally:
        h.lib.mr_destroy(h.ctx)


@pytest.mark.parametrize("ntheta,nr", [(96, 48), (256, 128)])
def test_library_own_locate_reproduces_receiver_positions(ntheta, nr):
    """The library's own search on a curvilinear donor (no inverse map given)
    inverts the donor's coordinates as interpolated by cubic Lagrange
    polynomials, the interpolation the cubic (width 4) stencils then apply:
    interpolating the donor's coordinates with a receiver's weights gives the
    receiver's position to rounding (Lagrange weights sum to one and
    reproduce the interpolant).  Against the closed-form inverse of the
    O-mesh's mapping, the weights differ only by the cubic interpolant's
    geometric error, which falls at fourth order with the O-mesh's spacing:
    the same donor points, weight differences below C * (1/ntheta)^4."""
    from paper_1805_06607_amd.system import HostSetup
    wl = workloads.cylinder(nbg=2 * ntheta, ntheta=ntheta, nr=nr)
    own = HostSetup(wl, own_locate=True)
    ref = HostSetup(wl)
    try:
        X = [gr.points() for gr in wl.grids]
        n_checked = 0
        for g in range(len(wl.grids)):
            assert np.array_equal(own.recv_order[g], ref.recv_order[g])
            for dg, (rr, pp, ww) in own.donor_tables[g].items():
                rr2, pp2, ww2 = ref.donor_tables[g][dg]
                assert np.array_equal(rr, rr2) and np.array_equal(pp, pp2)
                if wl.grids[dg].kind == workloads.CURVILINEAR:
                    xi = np.einsum("ks,dks->dk", ww, X[dg][:, pp])
                    err = np.max(np.abs(xi - X[g][:, rr]))
                    assert err < 1e-12, (g, dg, err)
                    dw = np.max(np.abs(ww - ww2))
                    assert 0 < dw < 0.1 * (100.0 / ntheta) ** 4, (g, dg, dw)
                    n_checked += len(rr)
                else:
                    assert np.array_equal(ww, ww2)
        assert n_checked > 30
    finally:
        own.lib.mr_destroy(own.ctx)
        ref.lib.mr_destroy(ref.ctx)


def test_assembly_errors():
    """A receiver no grid can serve and a failing locate callback are setup
    errors; receivers cannot be registered twice."""
    import ctypes
    from paper_1805_06607_amd import _lib
    from paper_1805_06607_amd.system import HostSetup
    wl = workloads.vortex_box()
    h = HostSetup(wl)
    lib = h.lib
    try:
        prio = (ctypes.c_int * 2)(0, 1)
        assert _lib.STATUS[lib.mr_assemble_overset(h.ctx, 4, prio, _lib.LOCATE_FN(), None)] == "MR_ERR_STATE"
        assert _lib.STATUS[lib.mr_assemble_overset(h.ctx, 3, prio, _lib.LOCATE_FN(), None)] == "MR_ERR_ARG"
    finally:
        lib.mr_destroy(h.ctx)
    # the background's hole grown past the patch: no receiver has a donor
    wl = workloads.vortex_box()
    c, hb = 5.0, 0.5 * 31 * (10.0 / 128) + 2 * (10.0 / 64)
    wl.grids[0].holes = [("box", (c - hb, c - hb), (c + hb, c + hb))]
    with pytest.raises(_lib.MrabError, match="without a donor"):
        HostSetup(wl)
    # a locate callback that fails
    wl = workloads.cylinder(nbg=128, ntheta=96, nr=48)
    wl.grids[1].inverse = None
    with pytest.raises(_lib.MrabError, match="locate callback failed"):
        HostSetup(wl)


@pytest.mark.parametrize("case", ["vortex_box", "cylinder_small", "tgv3d_small"])
def test_receiver_data_vectorised_equals_loop_bitwise(case):
    """The oracle's receiver data over all receivers at once takes each
    receiver's stencil sum in the same order as the receiver-by-receiver loop."""
    wl = {"vortex_box": lambda: workloads.vortex_box(),
          "cylinder_small": lambda: workloads.cylinder(nbg=96, ntheta=64, nr=32, half=6.0),
          "tgv3d_small": lambda: workloads.tgv3d(nbg=48, npatch=24, ninner=16)}[case]()
    s = OracleSystem(wl)
    states = workloads.random_state_like(wl, seed=9, amp=0.02)
    for g in range(len(wl.grids)):
        a = s.receiver_data(g, states)
        b = s.receiver_data_loop(g, states)
        assert np.array_equal(a, b)
