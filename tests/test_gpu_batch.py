"""Batched systems (C ABI mr_batch_*) against each system stepped on its own:
the same work-list kernels' per-tile and per-chunk code, so every system's
states and histories are bitwise those of its own macrosteps."""
import sys

import pytest

import workloads
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _systems(wls):
    from paper_1805_06607_amd.system import System
    out = []
    for wl in wls:
        s = System(wl)
        s.timestep()
        s.start(0.0)
        out.append(s)
    return out


def _snap(s):
    m = s.wl.params["hist_len"]
    return [s.state(g).clone() for g in range(s.ngrids)] + \
        [s.history(g, j).clone() for g in range(s.ngrids) for j in range(m)]


def test_batch_bitwise_equals_individual(torch):
    from paper_1805_06607_amd.batch import Batch
    wls = workloads.batch_vortex(6, seed=5, smin=24, smax=48)
    _say("systems", [(w.grids[0].n[0], w.grids[1].n[0], w.grids[1].rate) for w in wls])
    solo = _systems(wls)
    grouped = _systems(workloads.batch_vortex(6, seed=5, smin=24, smax=48))
    b = Batch(grouped)
    for n in (1, 5, 12, 7):
        b.macrostep(n)
        for s in solo:
            s.macrostep(n)
        torch.cuda.synchronize()
        for i, (a, c) in enumerate(zip(solo, grouped)):
            assert a.time() == c.time(), (n, i)
            for x, y in zip(_snap(a), _snap(c)):
                assert torch.equal(x, y), (n, i)
        _say("after", n, "macrosteps: bitwise equal")
    # a system stepped on its own in between: the batch rebuilds its plan
    solo[2].macrostep(3)
    grouped[2].macrostep(3)
    b.macrostep(4)
    for s in solo:
        s.macrostep(4)
    torch.cuda.synchronize()
    for a, c in zip(solo, grouped):
        for x, y in zip(_snap(a), _snap(c)):
            assert torch.equal(x, y)
    b.close()


def test_batch_rejects_unsupported(torch):
    from paper_1805_06607_amd import _lib
    from paper_1805_06607_amd.batch import Batch
    mixed = _systems([workloads.vortex_box(nbg=32, npatch=16),
                      workloads.cylinder(nbg=96, ntheta=64, nr=32, half=6.0)])
    with pytest.raises(_lib.MrabError):
        Batch(mixed)


def test_batch_common_tile_shape(torch):
    """With one tile shape for the whole batch, every system still equals its
    own macrosteps run with that shape."""
    from paper_1805_06607_amd.batch import Batch
    wls = workloads.batch_vortex(4, seed=7, smin=30, smax=60)
    solo = _systems(wls)
    for s in solo:
        for g in range(s.ngrids):
            s.set_tile_shape(g, 0)
    grouped = _systems(workloads.batch_vortex(4, seed=7, smin=30, smax=60))
    b = Batch(grouped)
    b.set_tile_shape(0)
    b.macrostep(9)
    for s in solo:
        s.macrostep(9)
    torch.cuda.synchronize()
    for a, c in zip(solo, grouped):
        for x, y in zip(_snap(a), _snap(c)):
            assert torch.equal(x, y)
    b.close()


def test_batch_systems_match_oracle_after_100_macrosteps(torch):
    """Three vortex systems of uneven size with patch rates 1, 2 and 4,
    advanced together for 100 macrosteps: each system's states against the
    oracle's own MRAB run of that system (relative L2 per variable over
    active points <= 1e-10)."""
    import numpy as np
    from gpu_util import rel_l2
    from oracle import OracleSystem
    from paper_1805_06607_amd.batch import Batch
    from paper_1805_06607_amd.system import System
    spacing = 10.0 / 64.0
    specs = [(40, 16, 1, (3.1, 3.3)), (48, 20, 2, (3.6, 3.9)), (56, 24, 4, (4.4, 4.0))]
    wls = [workloads.vortex_box(nbg=S, npatch=P, rate_patch=r, spacing=spacing, centre=c) for S, P, r, c in specs]
    orcs, systems = [], []
    for wl in wls:
        orc = OracleSystem(wl)
        _, H = orc.timestep()
        wl.params["dt_fixed"] = H
        orcs.append((orc, H))
        s = System(wl)
        s.timestep()
        s.start(0.0)
        systems.append(s)
    b = Batch(systems)
    b.macrostep(100)
    torch.cuda.synchronize()
    for i, (wl, (orc, H), s) in enumerate(zip(wls, orcs, systems)):
        mr = orc.integrator(H)
        mr.bootstrap(wl.q0)
        for _ in range(100):
            mr.macrostep()
        for g in range(len(wl.grids)):
            act = orc.grids[g].iblank.astype(bool)
            e = rel_l2(s.state(g).cpu().numpy(), mr.y[g], act)
            _say("batch vs oracle", i, "rate", wl.grids[1].rate, "grid", g, e)
            assert np.all(e <= 1e-10), (i, g, e)
    b.close()


def test_batch_autotune(torch):
    """The batch autotuner times every candidate, leaves every system's
    states, histories and time unchanged, and keeps the fastest shape, with
    which the batch still equals each system run alone with that shape."""
    from paper_1805_06607_amd.batch import Batch
    wls = workloads.batch_vortex(5, seed=11, smin=40, smax=96)
    grouped = _systems(wls)
    before = [_snap(s) for s in grouped]
    times = [s.time() for s in grouped]
    b = Batch(grouped)
    shape, ms = b.autotune(reps=3)
    torch.cuda.synchronize()
    _say("batch autotune pick", shape, {k: round(v, 4) for k, v in ms.items()})
    assert -1 <= shape < 8 and len(ms) == 9 and all(v > 0 for v in ms.values())
    assert ms[shape] == min(ms.values())
    for s, snap, t in zip(grouped, before, times):
        assert s.time() == t
        for x, y in zip(_snap(s), snap):
            assert torch.equal(x, y)
    solo = _systems(workloads.batch_vortex(5, seed=11, smin=40, smax=96))
    if shape >= 0:
        for s in solo:
            for g in range(s.ngrids):
                s.set_tile_shape(g, shape)
    b.macrostep(8)
    for s in solo:
        s.macrostep(8)
    torch.cuda.synchronize()
    for a, c in zip(solo, grouped):
        for x, y in zip(_snap(a), _snap(c)):
            assert torch.equal(x, y)
    b.close()
