"""Overset assembly for the product path (host, once per problem, untimed).

Section "SAT-Based Interpolation" of the paper lists the Chimera phases: grid
collision, hole cutting / fringe determination, donor-receiver search and
Lagrange interpolation with weights from Lagrange shape functions.  The
algorithms are those of a cited reference not reproduced in the paper; this
module implements the following rules with whole-array numpy operations:

* blanking: a point strictly inside one of its grid's hole shapes is a hole;
* receivers: active points that end a run of active points on an interface
  face (next to a hole, or on a grid face flagged as interface);
* donors: for each receiver, the first other grid in decreasing priority
  (ties: lowest grid id) whose W-point-per-direction stencil around the
  receiver's fractional index lies inside the grid (wrapping periodic
  directions) and covers only active points; stencil base floor(f) - (W/2-1);
  weights: tensor products of 1D Lagrange shape functions on W integer nodes,
  entry order x fastest.
"""
from __future__ import annotations

import numpy as np

BC_INTERFACE = 1


class SetupError(RuntimeError):
    pass


def iblank(grid) -> np.ndarray:
    X = grid.points()
    hole = np.zeros(grid.npts, dtype=bool)
    for shape in grid.holes:
        kind = shape[0]
        if kind == "box":
            lo = np.asarray(shape[1], dtype=float)[:, None]
            hi = np.asarray(shape[2], dtype=float)[:, None]
            hole |= np.all((X > lo) & (X < hi), axis=0)
        elif kind == "disk":
            c = np.asarray(shape[1], dtype=float)[:, None]
            hole |= np.sum((X - c) ** 2, axis=0) < shape[2] ** 2
        else:
            raise SetupError(f"unknown hole shape {kind!r}")
    return (~hole).astype(np.int8)


def receivers(grid, ib: np.ndarray) -> np.ndarray:
    dim = grid.dim
    A = ib.reshape(tuple(reversed(grid.n))).astype(bool)
    rec = np.zeros_like(A)
    for d in range(dim):
        ax = dim - 1 - d
        n = grid.n[d]
        idx = np.arange(n).reshape([-1 if a == ax else 1 for a in range(dim)])
        if grid.periodic[d]:
            before = np.roll(A, 1, axis=ax)
            after = np.roll(A, -1, axis=ax)
            start = A & ~before
            end = A & ~after
        else:
            before = np.roll(A, 1, axis=ax)
            after = np.roll(A, -1, axis=ax)
            lo_face = grid.face_bc[2 * d] == BC_INTERFACE
            hi_face = grid.face_bc[2 * d + 1] == BC_INTERFACE
            start = A & np.where(idx == 0, lo_face, ~before)
            end = A & np.where(idx == n - 1, hi_face, ~after)
        rec |= start | end
    return np.nonzero(rec.ravel())[0].astype(np.int64)


def lagrange_1d(s: np.ndarray, W: int) -> np.ndarray:
    """(K, W) Lagrange shape functions on nodes 0..W-1 at positions s (K,)."""
    out = np.ones((s.shape[0], W))
    nodes = np.arange(W, dtype=float)
    for a in range(W):
        for b in range(W):
            if b != a:
                out[:, a] *= (s - nodes[b]) / (nodes[a] - nodes[b])
    return out


def donors(grids, ibs, recvs, W: int):
    """Per receiving grid: dict donor grid -> (receiver points, donor points
    (K, S), weights (K, S))."""
    order = sorted(range(len(grids)), key=lambda k: (-grids[k].priority, k))
    out = []
    for g, grid in enumerate(grids):
        rp = recvs[g]
        X = grid.points()[:, rp]
        todo = np.ones(len(rp), dtype=bool)
        res = {}
        for dg in order:
            if dg == g or not todo.any():
                continue
            D = grids[dg]
            sel = np.nonzero(todo)[0]
            f = D.frac_index(X[:, sel])
            ok = np.all(np.isfinite(f), axis=0)
            base = np.floor(np.where(np.isfinite(f), f, 0.0)).astype(np.int64) - (W // 2 - 1)
            ids, wts = [], []
            for d in range(D.dim):
                a = base[d][:, None] + np.arange(W)[None, :]
                if D.periodic[d]:
                    a = np.mod(a, D.n[d])
                else:
                    ok &= (base[d] >= 0) & (base[d] + W - 1 <= D.n[d] - 1)
                    a = np.clip(a, 0, D.n[d] - 1)
                ids.append(a)
                wts.append(lagrange_1d(f[d] - base[d], W))
            S = W ** D.dim
            pts = np.zeros((len(sel), S), dtype=np.int64)
            w = np.ones((len(sel), S))
            stride = 1
            strides = []
            for d in range(D.dim):
                strides.append(stride)
                stride *= D.n[d]
            for e in range(S):
                for d in range(D.dim):
                    a = (e // W ** d) % W
                    pts[:, e] += ids[d][:, a] * strides[d]
                    w[:, e] *= wts[d][:, a]
            ok &= np.all(ibs[dg][pts] != 0, axis=1)
            hit = sel[ok]
            if len(hit):
                res[dg] = (rp[hit], pts[ok], w[ok])
                todo[hit] = False
        if todo.any():
            raise SetupError(f"grid {grid.name}: {int(todo.sum())} receivers without a donor")
        out.append(res)
    return out
