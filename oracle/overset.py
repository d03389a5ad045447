"""Overset assembly for the oracle: blanking, runs, receivers, donors, weights.

Part of the test oracle (test infrastructure only).

Paper: section "SAT-Based Interpolation" lists the Chimera phases (grid
collision, hole cutting / fringe determination, donor-receiver search, Lagrange
interpolation with weights from Lagrange shape functions); the algorithms
themselves live in a cited reference not included in the paper, so this module
follows these readings:

* A point is blanked when it lies strictly inside one of its grid's hole
  shapes (the shapes are part of the problem description).
* Each grid line, in each direction, splits into maximal runs of active points;
  a run may wrap across a periodic seam; a periodic line without holes has no
  ends.  Run ends carry a SAT face: at a grid face it is that face's boundary
  condition, next to a hole it is an interface.  Runs shorter than two
  closures are rejected.
* Receivers are the active points that end a run on an interface face.
* Donor: among the other grids, in decreasing priority (ties: lowest grid id),
  the first whose W-wide stencil (per direction) around the receiver's
  fractional index lies inside the grid and covers only active points.  The
  stencil base is floor(f) - (W/2 - 1); weights are tensor products of 1D
  Lagrange shape functions on the W integer nodes.
* The fractional index of a physical point in a donor grid is located here,
  not taken from the problem description's inverse map: on a Cartesian grid
  it is (x - origin) / spacing; on a curvilinear grid the nearest grid point
  (a scan over all coordinates) starts a Newton iteration on the grid's
  continuous mapping (whose integer samples are the grid's coordinates).
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from . import sbp as _sbp

BC_PERIODIC, BC_INTERFACE, BC_FARFIELD, BC_WALL = 0, 1, 2, 3


class AssemblyError(RuntimeError):
    pass


def blank(grid) -> np.ndarray:
    """iblank: 1 active, 0 hole."""
    X = grid.points()
    ib = np.ones(grid.npts, dtype=np.int8)
    for shape in grid.holes:
        if shape[0] == "box":
            lo, hi = shape[1], shape[2]
            inside = np.ones(grid.npts, dtype=bool)
            for d in range(grid.dim):
                inside &= (X[d] > lo[d]) & (X[d] < hi[d])
        elif shape[0] == "disk":
            c, r = shape[1], shape[2]
            rr = sum((X[d] - c[d]) ** 2 for d in range(grid.dim))
            inside = rr < r * r
        else:
            raise AssemblyError(f"unknown hole shape {shape[0]}")
        ib[inside] = 0
    return ib


def _strides(n):
    s = [1]
    for d in range(1, len(n)):
        s.append(s[-1] * n[d - 1])
    return s


def runs(grid, iblank: np.ndarray, sbp: int):
    """Per direction d: pos[d], rlen[d] (0: endless periodic line, -1: hole),
    bclo[d], bchi[d] (boundary flag at the start / end of the point's run)."""
    dim, n = grid.dim, grid.n
    nb = _sbp.nclosure(sbp)
    st = _strides(n)
    N = grid.npts
    out = []
    act = iblank.reshape(tuple(reversed(n)))   # [k][j][i]
    for d in range(dim):
        pos = np.full(N, -1, dtype=np.int32)
        rlen = np.full(N, -1, dtype=np.int32)
        bclo = np.zeros(N, dtype=np.int8)
        bchi = np.zeros(N, dtype=np.int8)
        nd = n[d]
        per = grid.periodic[d]
        # enumerate lines: every combination of the other indices
        others = [e for e in range(dim) if e != d]
        ranges = [range(n[e]) for e in others]
        import itertools
        for combo in itertools.product(*ranges):
            base = sum(c * st[e] for c, e in zip(combo, others))
            idx = [base + i * st[d] for i in range(nd)]
            a = [bool(iblank[p]) for p in idx]
            if all(a) and per:
                for i, p in enumerate(idx):
                    pos[p] = i
                    rlen[p] = 0
                continue
            if not any(a):
                continue
            # list runs as (start, length) in line coordinates (may wrap)
            line_runs = []
            if per:
                first_hole = a.index(False)
                i = 0
                while i < nd:
                    k = (first_hole + 1 + i) % nd
                    if a[k]:
                        s = k
                        L = 0
                        while i < nd and a[(first_hole + 1 + i) % nd]:
                            L += 1
                            i += 1
                        line_runs.append((s, L))
                    else:
                        i += 1
            else:
                i = 0
                while i < nd:
                    if a[i]:
                        s = i
                        while i < nd and a[i]:
                            i += 1
                        line_runs.append((s, i - s))
                    else:
                        i += 1
            for s, L in line_runs:
                if L < 2 * nb:
                    raise AssemblyError(
                        f"grid {grid.name}: run of {L} points along direction {d} "
                        f"is shorter than two closures ({2 * nb})")
                e = (s + L - 1) % nd
                lo = grid.face_bc[2 * d] if (not per and s == 0) else BC_INTERFACE
                hi = grid.face_bc[2 * d + 1] if (not per and e == nd - 1) else BC_INTERFACE
                for r in range(L):
                    p = idx[(s + r) % nd]
                    pos[p] = r
                    rlen[p] = L
                    bclo[p] = lo
                    bchi[p] = hi
        out.append((pos, rlen, bclo, bchi))
    return out


def receivers(grid, run_info) -> np.ndarray:
    """Flat indices (ascending) of active points ending a run on an interface face."""
    rec = []
    for p in range(grid.npts):
        is_rec = False
        for d in range(grid.dim):
            pos, rlen, bclo, bchi = run_info[d]
            if rlen[p] <= 0:
                continue
            if pos[p] == 0 and bclo[p] == BC_INTERFACE:
                is_rec = True
            if pos[p] == rlen[p] - 1 and bchi[p] == BC_INTERFACE:
                is_rec = True
        if is_rec:
            rec.append(p)
    return np.array(rec, dtype=np.int64)


def receivers_fast(grid, run_info) -> np.ndarray:
    """Same set as receivers(), computed with whole-array comparisons."""
    mask = np.zeros(grid.npts, dtype=bool)
    for d in range(grid.dim):
        pos, rlen, bclo, bchi = run_info[d]
        ok = rlen > 0
        mask |= ok & (pos == 0) & (bclo == BC_INTERFACE)
        mask |= ok & (pos == rlen - 1) & (bchi == BC_INTERFACE)
    return np.nonzero(mask)[0].astype(np.int64)


def lagrange_weights_1d(s: float, W: int) -> List[float]:
    """Lagrange shape functions on nodes 0..W-1 evaluated at s."""
    w = []
    for a in range(W):
        v = 1.0
        for b in range(W):
            if b != a:
                v *= (s - b) / (a - b)
        w.append(v)
    return w


def locate(grid, x: np.ndarray) -> np.ndarray:
    """Fractional index (dim,) of the physical point x (dim,) in grid; NaN
    components when it cannot be located (a curvilinear grid without a
    mapping, or a Newton iteration that does not converge)."""
    dim = grid.dim
    x = np.asarray(x, dtype=np.float64).reshape(dim)
    if grid.kind == 0:
        return np.array([(x[d] - grid.origin[d]) / grid.spacing[d] for d in range(dim)])
    if grid.mapping is None:
        return np.full(dim, np.nan)
    # start: the nearest grid point
    d2 = np.zeros(grid.npts)
    for d in range(dim):
        d2 += (grid.coords[d] - x[d]) ** 2
    p = int(np.argmin(d2))
    xi = np.zeros(dim)
    rest = p
    for d in range(dim):
        xi[d] = rest % grid.n[d]
        rest //= grid.n[d]
    # Newton on mapping(xi) = x with a central-difference Jacobian; the
    # residual is exact, so the Jacobian's error only slows convergence
    eps = 1e-6
    polish = None
    for _ in range(60):
        res = grid.mapping(xi[:, None])[:, 0] - x
        J = np.zeros((dim, dim))
        for e in range(dim):
            a = xi.copy()
            b = xi.copy()
            a[e] += eps
            b[e] -= eps
            J[:, e] = (grid.mapping(a[:, None])[:, 0] - grid.mapping(b[:, None])[:, 0]) / (2 * eps)
        try:
            step = np.linalg.solve(J, res)
        except np.linalg.LinAlgError:
            return np.full(dim, np.nan)
        xi = xi - step
        if not np.all(np.isfinite(xi)):
            return np.full(dim, np.nan)
        if polish is not None:
            polish -= 1
            if polish == 0:
                break
        elif np.max(np.abs(step)) < 1e-12:
            polish = 2          # two more steps at the rounding floor
    else:
        return np.full(dim, np.nan)
    if np.max(np.abs(grid.mapping(xi[:, None])[:, 0] - x)) > 1e-11 * (1.0 + np.max(np.abs(x))):
        return np.full(dim, np.nan)
    for d in range(dim):
        if grid.periodic[d]:
            xi[d] = xi[d] % grid.n[d]
    return xi


def donors(grids, iblanks, recv_lists, width: int):
    """For each receiving grid g: list of (donor grid id, point indices[W^dim],
    weights[W^dim]) in receiver order."""
    order = sorted(range(len(grids)), key=lambda k: (-grids[k].priority, k))
    result = []
    for g, grid in enumerate(grids):
        recs = recv_lists[g]
        X = grid.points()[:, recs] if len(recs) else np.zeros((grid.dim, 0))
        entries = []
        for r in range(len(recs)):
            x = X[:, r:r + 1]
            found = None
            for dg in order:
                if dg == g:
                    continue
                dgrid = grids[dg]
                f = locate(dgrid, x[:, 0])
                if not np.all(np.isfinite(f)):
                    continue
                idx1d, w1d, ok = [], [], True
                for d in range(dgrid.dim):
                    b = math.floor(f[d]) - (width // 2 - 1)
                    nd = dgrid.n[d]
                    if dgrid.periodic[d]:
                        ids = [(b + a) % nd for a in range(width)]
                    else:
                        if b < 0 or b + width - 1 > nd - 1:
                            ok = False
                            break
                        ids = [b + a for a in range(width)]
                    idx1d.append(ids)
                    w1d.append(lagrange_weights_1d(f[d] - b, width))
                if not ok:
                    continue
                st = _strides(dgrid.n)
                pts, wts = [], []
                for e in range(width ** dgrid.dim):
                    a = [(e // width ** d) % width for d in range(dgrid.dim)]
                    p = sum(idx1d[d][a[d]] * st[d] for d in range(dgrid.dim))
                    w = 1.0
                    for d in range(dgrid.dim):
                        w *= w1d[d][a[d]]
                    pts.append(p)
                    wts.append(w)
                if not all(iblanks[dg][p] for p in pts):
                    continue
                found = (dg, pts, wts)
                break
            if found is None:
                raise AssemblyError(f"grid {grid.name}: receiver {int(recs[r])} has no donor")
            entries.append(found)
        result.append(entries)
    return result
