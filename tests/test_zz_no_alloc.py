"""mr_bind_static_workspace: a system bound to the library's static
per-device workspace (no device allocation by the library or the binding)
computes what the same system bound to caller memory computes, for two systems
in a row on one device, the second smaller than the first; the first loses the
array to the second; a system larger than the array is refused before any
device work."""
import numpy as np
import pytest

import workloads
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def run(sysg, nmacro):
    """Right-hand side of a seeded state, then the bootstrap and nmacro
    macrosteps from the problem's initial state."""
    states = workloads.random_state_like(sysg.wl, seed=21, amp=0.02)
    F = [f.cpu().numpy() for f in sysg.rhs(states)]
    sysg.set_states(sysg.wl.q0)
    sysg.timestep()
    sysg.start(0.0)
    sysg.macrostep(nmacro)
    y = [sysg.state(g).cpu().numpy() for g in range(sysg.ngrids)]
    hist = [[sysg.history(g, j).cpu().numpy() for j in range(sysg.wl.params["hist_len"])]
            for g in range(sysg.ngrids)]
    return F, y, hist


def assert_same(a, b):
    for x, y in zip(a, b):
        if isinstance(x, list):
            assert_same(x, y)
        else:
            assert np.array_equal(x, y)


def test_static_workspace_matches_caller_workspace(torch):
    from paper_1805_06607_amd import _lib
    from paper_1805_06607_amd.system import System
    print("static workspace: vortex_box 64/32, then 48/24", flush=True)
    wl_a = workloads.vortex_box()
    wl_b = workloads.vortex_box(nbg=48, npatch=24)
    # first call: the larger system
    a_static = System(wl_a, static_workspace=True)
    a_ref = System(wl_a)
    assert a_static.workspace_bytes > System(wl_b).workspace_bytes
    got, want = run(a_static, 12), run(a_ref, 12)
    torch.cuda.synchronize()
    assert_same(got, want)
    # second call: a smaller system takes the array over
    b_static = System(wl_b, static_workspace=True)
    b_ref = System(wl_b)
    got, want = run(b_static, 9), run(b_ref, 9)
    torch.cuda.synchronize()
    assert_same(got, want)
    # the first system lost the array: its calls fail without touching it
    with pytest.raises(_lib.MrabError, match="bound to another context"):
        a_static.macrostep(1)
    # the holder keeps working after the failed call of the other context
    b_static.macrostep(3)
    b_ref.macrostep(3)
    for g in range(b_ref.ngrids):
        assert np.array_equal(b_static.state(g).cpu().numpy(), b_ref.state(g).cpu().numpy())
    a_static.close()
    b_static.close()


def test_static_workspace_refuses_large_system(torch):
    from paper_1805_06607_amd import _lib
    from paper_1805_06607_amd.system import System
    wl = workloads.vortex_box(nbg=256, npatch=128)
    with pytest.raises(_lib.MrabError, match="exceeds the static workspace"):
        System(wl, static_workspace=True)
