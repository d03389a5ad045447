"""GPU parity: the HIP path (through the C ABI) against the independent CPU
oracle, on the same seeded synthetic inputs.

Tolerances: one right-hand side, relative L2 per variable <= 1e-12 (the two
sides differ only in rounding order and FMA contraction); after 100 MRAB
macrosteps, relative L2 per variable <= 1e-10 over active points.
"""
import sys

import numpy as np
import pytest

import workloads
from gpu_util import rel_l2, require_gpu

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "vortex_box": lambda: workloads.vortex_box(),
    "cylinder_small": lambda: workloads.cylinder(nbg=96, ntheta=64, nr=32, half=6.0),
    # extended history (m = 6 > n = 4): more history values than a riding
    # launch's tiles park in LDS
    "cylinder_small_m6": lambda: workloads.cylinder(nbg=96, ntheta=64, nr=32, half=6.0, hist_len=6),
    "mms_box_42": lambda: workloads.mms_box(48, viscous=True, sbp=42),
    "torus_curvilinear": lambda: workloads.periodic_curvilinear(40, 36),
    "omesh_freestream": lambda: workloads.omesh_freestream(),
}


# donor data: one launch per link and donor step (chunked receivers, the
# default for 2D stencils) or values at distinct donor points, then a gather
DONOR_MODES = {"blocks": {}, "two_phase": {"donor_blocks": 0}}


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("two_pass", [0, 1])
@pytest.mark.parametrize("case", list(CASES))
def test_rhs_parity(torch, case, two_pass):
    """Fused tile kernel (default) and the gradient-pass form."""
    from oracle import OracleSystem
    from paper_1805_06607_amd.system import System
    wl = CASES[case]()
    _say("rhs parity", case, [g.n for g in wl.grids], "two_pass", two_pass)
    states = workloads.random_state_like(wl, seed=7, amp=0.02)
    orc = OracleSystem(wl)
    want = orc.rhs(states)
    sysg = System(wl)
    sysg.set_option("rhs_two_pass", two_pass)
    got = sysg.rhs(states)
    torch.cuda.synchronize()
    for g in range(len(wl.grids)):
        act = orc.grids[g].iblank.astype(bool)
        e = rel_l2(_np(got[g]), want[g], act)
        _say(case, g, e)
        assert np.all(e <= 1e-12), (case, g, e)
        assert np.all(_np(got[g])[:, ~act] == 0.0)


@pytest.mark.parametrize("mode", list(DONOR_MODES))
@pytest.mark.parametrize("case", ["vortex_box", "cylinder_small"])
def test_receiver_data_parity(torch, case, mode):
    from oracle import OracleSystem
    from paper_1805_06607_amd.system import System
    wl = CASES[case]()
    states = workloads.random_state_like(wl, seed=3, amp=0.02)
    orc = OracleSystem(wl)
    sysg = System(wl)
    for name, value in DONOR_MODES[mode].items():
        sysg.set_option(name, value)
    for g in range(len(wl.grids)):
        want = orc.receiver_data(g, states)
        got = _np(sysg.receiver_data(g, states))
        assert got.shape == want.shape
        e = rel_l2(got.T, want.T)
        _say(case, g, "receiver data", e)
        assert np.all(e <= 1e-13), e


@pytest.mark.parametrize("case", ["vortex_box", "cylinder_small"])
def test_timestep_parity(torch, case):
    from oracle import OracleSystem
    from paper_1805_06607_amd.system import System
    wl = CASES[case]()
    orc = OracleSystem(wl)
    h0, H0 = orc.timestep()
    h1, H1 = System(wl).timestep()
    assert abs(H1 - H0) <= 1e-14 * H0 and abs(h1 - h0) <= 1e-14 * h0


def _run_both(wl, nmacro, options=None):
    from oracle import OracleSystem
    from paper_1805_06607_amd.system import System
    orc = OracleSystem(wl)
    h, H = orc.timestep()
    wl.params["dt_fixed"] = H           # both sides step with the same H
    mr = orc.integrator(H)
    mr.bootstrap(wl.q0)
    sysg = System(wl)
    for name, value in (options or {}).items():
        sysg.set_option(name, value)
    sysg.timestep()
    sysg.start(0.0)
    for k in range(nmacro):
        mr.macrostep()
    sysg.macrostep(nmacro)
    return orc, mr, sysg


@pytest.mark.parametrize("mode", list(DONOR_MODES))
@pytest.mark.parametrize("case", ["vortex_box", "cylinder_small", "cylinder_small_m6"])
def test_mrab_parity_100_macrosteps(torch, case, mode):
    wl = CASES[case]()
    _say("mrab parity", case, mode)
    orc, mr, sysg = _run_both(wl, 100, DONOR_MODES[mode])
    t, k = sysg.time()
    assert k == 100 and abs(t - mr.t) <= 1e-12 * mr.t
    for g in range(len(wl.grids)):
        act = orc.grids[g].iblank.astype(bool)
        e = rel_l2(_np(sysg.state(g)), mr.y[g], act)
        _say(case, g, "after 100 macrosteps", e)
        assert np.all(e <= 1e-10), (case, g, e)


@pytest.mark.parametrize("case", ["vortex_box", "cylinder_small"])
def test_fine_step_single_rate_reference(torch, case):
    """The equal-error protocol's reference run is single-rate AB at a
    32nd of the fast step: the same run on the GPU and in the oracle
    (every grid at h/32, 128 steps after the bootstrap) agree to 1e-10."""
    wl = CASES[case]()
    for g in wl.grids:
        g.rate = 1
    from oracle import OracleSystem
    h, _ = OracleSystem(CASES[case]()).timestep()
    wl.params["dt_fixed"] = h / 32
    _say("fine-step single-rate reference", case, h / 32)
    orc, mr, sysg = _run_both(wl, 128)
    for g in range(len(wl.grids)):
        act = orc.grids[g].iblank.astype(bool)
        e = rel_l2(_np(sysg.state(g)), mr.y[g], act)
        _say(case, g, "single-rate at h/32", e)
        assert np.all(e <= 1e-10), (case, g, e)


def test_bootstrap_history_parity(torch):
    wl = CASES["vortex_box"]()
    orc, mr, sysg = _run_both(wl, 0)
    for g in range(len(wl.grids)):
        act = orc.grids[g].iblank.astype(bool)
        for j in range(wl.params["hist_len"]):
            e = rel_l2(_np(sysg.history(g, j)), mr.hist[g][j], act)
            assert np.all(e <= 1e-11), (g, j, e)


def test_ratio_one_is_single_rate_ab_bitwise(torch):
    """MRAB with every rate equal reproduces, bit for bit, a single-rate AB
    loop assembled from mr_rhs and separately rounded products and sums."""
    from paper_1805_06607_amd.system import System, ab_coeffs
    wl = workloads.vortex_box(rate_bg=1, rate_patch=1)
    sysg = System(wl)
    h, H = sysg.timestep()
    sysg.start(0.0)
    m = wl.params["hist_len"]
    y = [sysg.state(g).clone() for g in range(2)]
    hist = [[sysg.history(g, j).clone() for j in range(m)] for g in range(2)]
    c = [float(a) * H for a in ab_coeffs(wl.params["order"], m, 1.0)]
    N = 20
    for _ in range(N):
        for g in range(2):
            acc = y[g].clone()
            for j in range(m):
                acc = acc + (c[j] * hist[g][j])
            y[g] = acc
        F = sysg.rhs(y)
        F = [f.clone() for f in F]
        for g in range(2):
            hist[g] = hist[g][1:] + [F[g]]
    sysg.macrostep(N)
    torch.cuda.synchronize()
    for g in range(2):
        assert torch.equal(sysg.state(g), y[g]), g


def test_determinism_bitwise(torch):
    from paper_1805_06607_amd.system import System
    outs = []
    for _ in range(2):
        wl = CASES["cylinder_small"]()
        s = System(wl)
        s.timestep()
        s.start(0.0)
        s.macrostep(10)
        outs.append([s.state(g).clone() for g in range(2)])
    for g in range(2):
        assert torch.equal(outs[0][g], outs[1][g])


def test_mrab_parity_full_size_cylinder(torch):
    """The benchmark workload itself (512^2 background + 256x128 O-mesh, AB4,
    ratio 4): 100 macrosteps, GPU vs oracle."""
    wl = workloads.cylinder()
    _say("mrab parity full-size cylinder")
    orc, mr, sysg = _run_both(wl, 100)
    for g in range(len(wl.grids)):
        act = orc.grids[g].iblank.astype(bool)
        e = rel_l2(_np(sysg.state(g)), mr.y[g], act)
        _say("cylinder full", g, e)
        assert np.all(e <= 1e-10), (g, e)


def test_tile_shapes_agree(torch):
    """Every tile shape of the fused 2D kernel gives the same result up to
    rounding (the compiler may contract a multiply-add differently per
    instantiation): one right-hand side on ragged curvilinear grids, and 5
    MRAB macrosteps of the small cylinder case (set explicitly and as picked
    by the autotuner)."""
    from paper_1805_06607_amd.system import System
    for case in ("torus_curvilinear", "omesh_freestream"):
        wl = CASES[case]()
        states = workloads.random_state_like(wl, seed=11, amp=0.02)
        ref = None
        for shape in range(-1, 8):
            s = System(wl)
            for g in range(len(wl.grids)):
                s.set_tile_shape(g, shape)
            out = [_np(f) for f in s.rhs(states)]
            if ref is None:
                ref = out
            for g in range(len(wl.grids)):
                e = rel_l2(out[g], ref[g])
                _say(case, "shape", shape, g, e)
                assert np.all(e <= 1e-13), (case, shape, g, e)
    ref = None
    for shape in list(range(-1, 8)) + ["auto"]:
        wl = CASES["cylinder_small"]()
        s = System(wl)
        s.timestep()
        if shape == "auto":
            _say("autotuned", s.autotune(reps=3))
        else:
            for g in range(2):
                s.set_tile_shape(g, shape)
        s.start(0.0)
        s.macrostep(5)
        out = [_np(s.state(g)) for g in range(2)]
        if ref is None:
            ref = out
        for g in range(2):
            e = rel_l2(out[g], ref[g])
            _say("cylinder_small shape", shape, g, e)
            assert np.all(e <= 1e-12), (shape, g, e)


@pytest.mark.parametrize("case", ["vortex_box", "cylinder_small"])
def test_multi_stream_bitwise(torch, case):
    """Per-grid streams ordered by events give the same bits as every launch
    in order on one stream.  The calls mix lengths, with host reads and
    synchronisation between them; every call's result is compared."""
    from paper_1805_06607_amd.system import System
    plans = {"one_stream": {"multi_stream": 0}, "streams": {"multi_stream": 1}}
    systems = {}
    for name, opts in plans.items():
        wl = CASES[case]()
        s = System(wl)
        for o, v in opts.items():
            s.set_option(o, v)
        s.timestep()
        s.start(0.0)
        systems[name] = s
    ng = len(wl.grids)
    m = wl.params["hist_len"]
    for n in (1, 7, 12, 5, 6, 13, 24):
        snap = {}
        for name, s in systems.items():
            s.macrostep(n)
            torch.cuda.synchronize()
            snap[name] = [s.state(g).clone() for g in range(ng)] + \
                [s.history(g, j).clone() for g in range(ng) for j in range(m)]
        for a, b in zip(snap["one_stream"], snap["streams"]):
            assert torch.equal(a, b), (case, n)
        t = [s.time() for s in systems.values()]
        assert t[0] == t[1], t


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["vortex_box", "cylinder_small", "cylinder_small_m6"])
@pytest.mark.parametrize("host_shape", [None, 1])
def test_ride_donors_bitwise(torch, case, host_shape):
    """A slow grid's mid-step donor data launched inside the next same-time
    grid's right-hand side (one launch less) gives the same bits as its own
    launch.  host_shape 1 (16 x 8 tiles, 128 threads) is too small to carry
    it, so that run checks the fallback to separate launches."""
    from paper_1805_06607_amd.system import System
    systems = {}
    for name, ride in (("separate", 0), ("riding", 1)):
        wl = CASES[case]()
        s = System(wl)
        s.set_option("multi_stream", 0)
        s.set_option("ride_donors", ride)
        if host_shape is not None:
            s.set_tile_shape(1, host_shape)
        s.timestep()
        s.start(0.0)
        systems[name] = s
    ng = len(wl.grids)
    m = wl.params["hist_len"]
    for n in (1, 3, 8):
        snap = {}
        for name, s in systems.items():
            s.macrostep(n)
            torch.cuda.synchronize()
            snap[name] = [s.state(g).clone() for g in range(ng)] + \
                [s.history(g, j).clone() for g in range(ng) for j in range(m)]
        for a, b in zip(snap["separate"], snap["riding"]):
            assert torch.equal(a, b), (case, host_shape, n)


@pytest.mark.skip(reason="graph replay of captured macrosteps is switched off: both runs of the "
                         "capture path ended the process with a segmentation fault inside the HIP "
                         "runtime; cause not found")
def test_graph_replay_bitwise(torch):
    from paper_1805_06607_amd.system import System
    wl = CASES["cylinder_small"]()
    ref, s = System(wl), System(CASES["cylinder_small"]())
    ref.set_option("multi_stream", 0)
    s.set_option("graph", 1)
    for x in (ref, s):
        x.timestep()
        x.start(0.0)
    for n in (1, 7, 12, 5):
        ref.macrostep(n)
        s.macrostep(n)
        torch.cuda.synchronize()
        for g in range(2):
            assert torch.equal(ref.state(g), s.state(g)), (n, g)
