"""Checkpoint and restart through the C ABI (mr_save / mr_load): the
macrosteps after a restart repeat those after the checkpoint bit for bit, in
the same context and in a fresh one built from the same problem."""
import numpy as np
import pytest

import workloads
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.mark.parametrize("case", ["vortex_box", "cylinder_small"])
def test_save_load_bitwise(torch, case):
    from paper_1805_06607_amd.system import System
    wl = workloads.vortex_box() if case == "vortex_box" else workloads.cylinder(nbg=96, ntheta=64, nr=32,
                                                                                  half=6.0)
    a = System(wl)
    a.timestep()
    a.start(0.0)
    a.macrostep(5)
    ck = a.save()
    t0, k0 = a.time()
    a.macrostep(7)
    want = [a.state(g).cpu().numpy() for g in range(a.ngrids)]
    want_t = a.time()
    # same context, restarted
    a.load(ck)
    assert a.time() == (t0, k0)
    a.macrostep(7)
    for g in range(a.ngrids):
        assert np.array_equal(a.state(g).cpu().numpy(), want[g])
    assert a.time() == want_t
    # a fresh context of the same problem (no mr_mrab_start)
    b = System(wl)
    b.load(ck)
    b.macrostep(7)
    for g in range(b.ngrids):
        assert np.array_equal(b.state(g).cpu().numpy(), want[g])
        for j in range(wl.params["hist_len"]):
            assert np.array_equal(b.history(g, j).cpu().numpy(), a.history(g, j).cpu().numpy())
    assert b.time() == want_t


def test_load_rejects_other_problem(torch):
    from paper_1805_06607_amd import _lib
    from paper_1805_06607_amd.system import System
    a = System(workloads.vortex_box())
    a.timestep()
    a.start(0.0)
    ck = a.save()
    b = System(workloads.cylinder(nbg=96, ntheta=64, nr=32, half=6.0))
    with pytest.raises(_lib.MrabError):
        b.load(ck)
    with pytest.raises(_lib.MrabError):
        a.load(ck[:100])


def test_load_rejects_same_size_other_problem(torch):
    """Checkpoints of problems with the same grids and point counts but
    another rate or another scheme are refused (the header records the
    scheme and every grid's sizes and rate)."""
    from paper_1805_06607_amd import _lib
    from paper_1805_06607_amd.system import System
    a = System(workloads.vortex_box(rate_patch=2))
    a.timestep()
    a.start(0.0)
    ck = a.save()
    # same grids, other patch rate
    with pytest.raises(_lib.MrabError, match="different problem"):
        System(workloads.vortex_box(rate_patch=4)).load(ck)
    # same grids, rates and history length, other order (AB2 on 3 values)
    w = workloads.vortex_box(rate_patch=2)
    w.params["order"] = 2
    with pytest.raises(_lib.MrabError, match="different problem"):
        System(w).load(ck)
    # the same problem loads
    b = System(workloads.vortex_box(rate_patch=2))
    b.load(ck)
    assert b.time() == a.time()
