"""Hole cutting for the product path (host, once per problem, untimed).

Section "SAT-Based Interpolation" of the paper lists the Chimera phases: grid
collision, hole cutting / fringe determination, donor-receiver search and
Lagrange interpolation with weights from Lagrange shape functions.  The
algorithms are those of a cited reference not reproduced in the paper.  The
problem description carries each grid's hole shapes; this module blanks the
points strictly inside one of them (the iblank array handed to the library).
Runs, fringe (receiver) points, the donor-receiver search and the Lagrange
weights are the library's (mr_add_grid, mr_assemble_overset).
"""
from __future__ import annotations

import numpy as np


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
