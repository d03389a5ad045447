"""Writes tgv3d_mrab100_samples.npz: the oracle's states of the full-size 3D
three-level problem (192^3 background, two 96^3 patches, 64^3 inner patch;
rates 1, 2, 2, 4; SBP 4-2, cubic donors, AB3) after the RK3 bootstrap and 100
MRAB macrosteps at the oracle's own macrostep H (CFL 0.4), at 3000 seeded
active points per grid, half of them within three points of a hole, an
interface face or a grid edge.  Calls only the oracle and the problem
description.  Run from the repository root: python tests/golden/make_tgv3d_samples.py
(about 40 minutes on 8 cores)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import OracleSystem  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tgv3d_mrab100_samples.npz")
NMACRO = 100


def near_boundary(ib, n, reach=3):
    act = np.asarray(ib).astype(bool).reshape(n[2], n[1], n[0])
    near = np.zeros_like(act)
    for ax in range(3):
        for s in range(1, reach + 1):
            near |= np.roll(~act, s, axis=ax) | np.roll(~act, -s, axis=ax)
        idx = [slice(None)] * 3
        idx[ax] = slice(0, reach)
        near[tuple(idx)] = True
        idx[ax] = slice(act.shape[ax] - reach, None)
        near[tuple(idx)] = True
    return np.flatnonzero((near & act).ravel())


def main():
    t0 = time.time()
    wl = workloads.tgv3d()
    orc = OracleSystem(wl)
    h, H = orc.timestep()
    print(f"setup {time.time() - t0:.0f} s, H = {H!r}", flush=True)
    mr = orc.integrator(H)
    mr.bootstrap(wl.q0)
    print(f"bootstrap done {time.time() - t0:.0f} s", flush=True)
    for k in range(NMACRO):
        mr.macrostep()
        print(f"macrostep {k + 1} {time.time() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(7)
    out = {"H": np.float64(H), "t": np.float64(mr.t), "nmacro": np.int64(NMACRO)}
    for g, gr in enumerate(wl.grids):
        ib = orc.grids[g].iblank
        act = np.flatnonzero(ib)
        nb = near_boundary(ib, gr.n)
        pts = np.unique(np.concatenate([rng.choice(act, 1500, replace=False),
                                        rng.choice(nb, min(1500, nb.size), replace=False)]))
        out[f"pts{g}"] = pts.astype(np.int64)
        out[f"q{g}"] = np.ascontiguousarray(mr.y[g][:, pts])
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
