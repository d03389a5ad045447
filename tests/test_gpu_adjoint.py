"""Discrete adjoint on the GPU (through the C ABI) against directional
derivatives of the oracle's forward map and of the library's own forward
pass, on seeded synthetic inputs.

Directional derivatives are central differences with one Richardson step
(error O(h^4) plus rounding ~1e-16 |f| / h); at the steps used here they are
good to about 1e-10 relative, so the adjoint's dot products are held to
1e-8 (right-hand side) and 1e-7 (whole runs, whose objective sums many
terms).  The checkpointing schedule only changes which forward macrosteps
are recomputed, so gradients are bitwise equal for every snapshot count.
"""
import sys

import numpy as np
import pytest

import workloads
from gpu_util import require_gpu

pytestmark = pytest.mark.gpu

CASES = {
    "vortex_box": lambda: workloads.vortex_box(),
    "cylinder_small": lambda: workloads.cylinder(nbg=96, ntheta=64, nr=32, half=6.0),
    "mms_box_42": lambda: workloads.mms_box(48, viscous=True, sbp=42),
    "torus_curvilinear": lambda: workloads.periodic_curvilinear(40, 36),
}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


def _np(t):
    return t.detach().cpu().numpy()


def _base(wl, seed, amp=0.02):
    """Seeded states near the workload's initial ones with every velocity
    component perturbed too: the SAT flux splitting takes |eigenvalue|, which
    is not differentiable where a normal velocity is exactly zero (as on the
    axis-aligned faces of a flow with v = 0), so derivatives are compared away
    from such states."""
    rng = np.random.default_rng(seed)
    out = []
    for q in workloads.random_state_like(wl, seed=seed, amp=amp):
        q = np.asarray(q, dtype=np.float64).reshape(wl.dim + 2, -1).copy()
        for i in range(wl.dim):
            q[1 + i] += amp * q[0] * rng.uniform(-1.0, 1.0, q.shape[1])
        out.append(q)
    return out


def _dirs(states, seed, n):
    """n seeded directions, each entry scaled by its state's magnitude."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        out.append([rng.standard_normal(s.shape) * np.abs(s) for s in states])
    return out


def _objective(case, wl, sysg):
    from paper_1805_06607_amd.adjoint import wall_objective
    if case == "cylinder_small":
        pts, w = wall_objective(wl.grids[1])
        return 1, pts, w
    g = len(wl.grids) - 1
    rng = np.random.default_rng(11)
    act = np.flatnonzero(sysg.iblanks[g])
    pts = np.sort(rng.choice(act, size=min(40, len(act)), replace=False))
    return g, pts, rng.uniform(0.5, 1.5, size=len(pts))


@pytest.mark.parametrize("case", list(CASES))
def test_adj_rhs_dot_products_vs_oracle(torch, case):
    """<w, J v> (oracle, finite differences) = <J^T w, v> (GPU adjoint) for
    the coupled right-hand side, on whole fields and on sampled unit
    directions (points at walls, far-field faces, interface receivers, donor
    points and the interior)."""
    from oracle import OracleSystem
    from oracle.adjoint import rhs_directional
    from paper_1805_06607_amd.adjoint import Adjoint
    from paper_1805_06607_amd.system import System
    wl = CASES[case]()
    _say("adjoint rhs", case, [g.n for g in wl.grids])
    states = _base(wl, 5)
    orc = OracleSystem(wl)
    sysg = System(wl)
    adj = Adjoint(sysg, nsnap=1)
    rng = np.random.default_rng(9)
    for trial, v in enumerate(_dirs(states, 21, 3)):
        w = [rng.standard_normal(s.shape) for s in states]
        jv = rhs_directional(orc, states, v, 1e-4)
        gt = [_np(a) for a in adj.rhs_vjp(states, w)]
        lhs = sum(float(np.sum(a * b)) for a, b in zip(w, jv))
        rhs = sum(float(np.sum(a * b)) for a, b in zip(gt, v))
        scale = sum(float(np.sum(np.abs(a * b))) for a, b in zip(w, jv))
        _say(case, trial, lhs, rhs, abs(lhs - rhs) / scale)
        assert abs(lhs - rhs) <= 1e-8 * scale, (case, trial, lhs, rhs)
    # sampled entries of J^T w: <w, J e_i>
    w = [rng.standard_normal(s.shape) for s in states]
    gt = [_np(a) for a in adj.rhs_vjp(states, w)]
    nv = wl.dim + 2
    picks = []
    for g, gr in enumerate(orc.grids):
        act = np.flatnonzero(gr.iblank)
        cls = []
        rp = np.asarray(sysg.recv_pts[g], dtype=np.int64)
        if len(rp):
            cls.append(rp[rng.integers(len(rp))])
        for tab in sysg.donor_tables:
            for dg, (_, dpts, _) in tab.items():
                if dg == g:
                    cls.append(int(np.asarray(dpts).ravel()[rng.integers(np.asarray(dpts).size)]))
        cls.append(int(act[0]))
        cls.append(int(act[rng.integers(len(act))]))
        for p in cls:
            picks.append((g, int(rng.integers(nv)), int(p)))
    for (g, v_, p) in picks:
        e = [np.zeros_like(s) for s in states]
        e[g][v_, p] = max(abs(states[g][v_, p]), 1e-3)
        jv = rhs_directional(orc, states, e, 1e-4)
        want = sum(float(np.sum(a * b)) for a, b in zip(w, jv)) / e[g][v_, p]
        got = gt[g][v_, p]
        _say(case, "entry", g, v_, p, got, want)
        assert abs(got - want) <= 1e-7 * max(abs(want), 1e-3 * np.max(np.abs(gt[g]))), (g, v_, p, got, want)


@pytest.mark.parametrize("case", ["vortex_box", "cylinder_small"])
def test_adj_forward_matches_macrosteps(torch, case):
    """The forward pass the adjoint differentiates is the method's run:
    its final states equal mr_mrab_start + mr_mrab_macrostep to rounding."""
    from paper_1805_06607_amd.adjoint import Adjoint
    from paper_1805_06607_amd.system import System
    wl = CASES[case]()
    sysg = System(wl)
    sysg.timestep()
    y0 = [np.asarray(q, dtype=np.float64).reshape(wl.dim + 2, -1) for q in wl.q0]
    adj = Adjoint(sysg, nsnap=2)
    _, yN = adj.forward(6, y0)
    sysg.set_states(y0)
    sysg.start(0.0)
    sysg.macrostep(6)
    for g in range(len(wl.grids)):
        a, b = _np(yN[g]), _np(sysg.state(g))
        e = np.max(np.abs(a - b)) / np.max(np.abs(b))
        _say(case, g, "forward vs macrosteps", e)
        assert e <= 1e-12


@pytest.mark.parametrize("case", ["vortex_box", "cylinder_small"])
def test_adj_gradient_vs_finite_differences(torch, case):
    """Whole-run gradient (bootstrap + MRAB macrosteps, checkpointed)
    against central differences of the GPU forward pass on seeded
    directions, and of the oracle's own run on two of them."""
    from oracle import OracleSystem
    from oracle.adjoint import richardson, run_objective
    from paper_1805_06607_amd.adjoint import Adjoint
    from paper_1805_06607_amd.system import System
    wl = CASES[case]()
    sysg = System(wl)
    h, H = sysg.timestep()
    nmacro = 4
    adj = Adjoint(sysg, nsnap=3)
    og, pts, w = _objective(case, wl, sysg)
    adj.set_objective(og, pts, w)
    y0 = _base(wl, 8, amp=0.01)
    J, grads, nf = adj.gradient(nmacro, y0)
    grads = [_np(g) for g in grads]
    _say(case, "J", J, "forward macrosteps", nf)
    orc = OracleSystem(wl)
    J_or, _ = run_objective(orc, y0, nmacro, H, og, pts, w)
    _say(case, "J oracle", J_or)
    assert abs(J - J_or) <= 1e-11 * abs(J_or)
    for k, v in enumerate(_dirs(y0, 31, 4)):
        got = sum(float(np.sum(a * b)) for a, b in zip(grads, v))
        fd = richardson(lambda e: adj.forward(nmacro, [y + e * d for y, d in zip(y0, v)])[0], 1e-4)
        _say(case, k, "adjoint", got, "fd", fd)
        assert abs(got - fd) <= 1e-7 * abs(fd), (k, got, fd)
        if k < 2:
            fdo = richardson(lambda e: run_objective(orc, [y + e * d for y, d in zip(y0, v)], nmacro, H, og, pts,
                                                     w)[0], 1e-4)
            _say(case, k, "oracle fd", fdo)
            assert abs(got - fdo) <= 1e-7 * abs(fdo), (k, got, fdo)


def test_adj_checkpointing_bitwise(torch):
    """Every snapshot count gives the same gradient bit for bit; the
    forward macrosteps run are the first pass plus the schedule's count."""
    from paper_1805_06607_amd.adjoint import Adjoint, schedule_cost, wall_objective
    from paper_1805_06607_amd.system import System
    wl = CASES["cylinder_small"]()
    y0 = _base(wl, 4, amp=0.01)
    pts, w = wall_objective(wl.grids[1])
    nmacro = 9
    ref = None
    for nsnap in (10, 1, 2, 3):
        sysg = System(wl)
        sysg.timestep()
        adj = Adjoint(sysg, nsnap=nsnap)
        adj.set_objective(1, pts, w)
        J, g, nf = adj.gradient(nmacro, y0)
        g = [_np(x) for x in g]
        _say("nsnap", nsnap, "J", J, "forward macrosteps", nf)
        assert nf == nmacro + schedule_cost(nmacro, nsnap)
        if ref is None:
            ref = (J, g)
        else:
            assert J == ref[0]
            for a, b in zip(g, ref[1]):
                assert np.array_equal(a, b)
        sysg.close()


def test_autograd_function(torch):
    """MRABRun inside a torch graph: the gradient of a loss mixing J and the
    final states, through an initial condition built with torch ops, equals
    the library's gradient with the same terminal adjoint (chain rule done
    by torch on the initial-condition map)."""
    from paper_1805_06607_amd.adjoint import Adjoint, MRABRun
    from paper_1805_06607_amd.system import System
    wl = CASES["vortex_box"]()
    sysg = System(wl)
    sysg.timestep()
    adj = Adjoint(sysg, nsnap=2)
    g, pts, w = _objective("vortex_box", wl, sysg)
    adj.set_objective(g, pts, w)
    dev = sysg.device
    base = [torch.as_tensor(np.asarray(q, dtype=np.float64).reshape(wl.dim + 2, -1), device=dev) for q in wl.q0]
    s = torch.ones((), dtype=torch.float64, device=dev, requires_grad=True)
    y0 = [b * s for b in base]
    out = MRABRun.apply(adj, 3, *y0)
    J, yN = out[0], out[1:]
    rng = np.random.default_rng(2)
    cs = [torch.as_tensor(rng.standard_normal(tuple(y.shape)), device=dev) for y in yN]
    loss = 2.5 * J + sum((c * y).sum() for c, y in zip(cs, yN))
    loss.backward()
    _, grads, _ = adj.gradient(3, [b.detach() for b in base], lamN=cs, jscale=2.5)
    want = sum(float((gr * b).sum()) for gr, b in zip(grads, base))
    _say("autograd", float(s.grad), want)
    assert float(s.grad) == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("nmacro", [0, 3])
def test_adj_terminal_adjoint_without_objective(torch, nmacro):
    """With no objective the gradient is that of <c, y_N> alone (nmacro = 0:
    the bootstrap only), against central differences of the forward pass."""
    from oracle.adjoint import richardson
    from paper_1805_06607_amd.adjoint import Adjoint
    from paper_1805_06607_amd.system import System
    wl = CASES["vortex_box"]()
    sysg = System(wl)
    sysg.timestep()
    adj = Adjoint(sysg, nsnap=2)
    y0 = _base(wl, 12, amp=0.01)
    rng = np.random.default_rng(5)
    cs = [rng.standard_normal(y.shape) for y in y0]
    J, grads, _ = adj.gradient(nmacro, y0, lamN=cs, jscale=0.0)
    assert J == 0.0
    grads = [_np(g) for g in grads]
    for k, v in enumerate(_dirs(y0, 41, 2)):
        got = sum(float(np.sum(a * b)) for a, b in zip(grads, v))

        def f(e):
            _, yN = adj.forward(nmacro, [y + e * d for y, d in zip(y0, v)])
            return sum(float(np.sum(c * _np(y))) for c, y in zip(cs, yN))

        fd = richardson(f, 1e-4)
        _say("terminal", nmacro, k, got, fd)
        assert abs(got - fd) <= 1e-7 * abs(fd)


TINY = {
    "vortex_box_21": lambda: workloads.vortex_box(nbg=20, npatch=14, Re=100.0),
    "cylinder_42": lambda: workloads.cylinder(nbg=40, ntheta=32, nr=12, half=6.0),
    "wall_channel_42": lambda: workloads.wall_channel(12),
}


@pytest.mark.parametrize("case", list(TINY))
def test_adj_rhs_whole_field_vs_dense_jacobian(torch, case):
    """J^T w of the GPU adjoint against the transpose of the oracle's dense
    Jacobian (central differences with one Richardson step, one column per
    active state entry), entry
    by entry over every grid: interfaces with bilinear and cubic donors,
    periodic seams, far-field faces, isothermal walls on the O-mesh and on
    Cartesian faces, curvilinear metrics."""
    from oracle import OracleSystem
    from paper_1805_06607_amd.adjoint import Adjoint
    from paper_1805_06607_amd.system import System
    wl = TINY[case]()
    states = _base(wl, 7)
    orc = OracleSystem(wl)
    sysg = System(wl)
    adj = Adjoint(sysg, nsnap=1)
    rng = np.random.default_rng(17)
    w = [rng.standard_normal(s.shape) for s in states]
    got = [_np(a) for a in adj.rhs_vjp(states, w)]
    nv = wl.dim + 2
    want = [np.zeros_like(s) for s in states]
    # step scale per variable: the momentum components share the largest
    # momentum magnitude (a nearly zero component would otherwise get a step
    # so small that rounding swamps the difference)
    scale = []
    for st in states:
        sc = np.max(np.abs(st), axis=1)
        sc[1:nv - 1] = np.max(sc[1:nv - 1])
        scale.append(sc)
    ncol = 0
    for g, gr in enumerate(orc.grids):
        act = np.flatnonzero(gr.iblank)
        for v in range(nv):
            for p in act:
                h = 1e-4 * max(abs(states[g][v, p]), scale[g][v])

                def central(hh):
                    plus = [s.copy() for s in states]
                    minus = [s.copy() for s in states]
                    plus[g][v, p] += hh
                    minus[g][v, p] -= hh
                    fp, fm = orc.rhs(plus), orc.rhs(minus)
                    return sum(float(np.sum(w[k] * (fp[k] - fm[k]))) for k in range(len(states))) / (2 * hh)

                # one Richardson step: error O(h^4) plus rounding
                want[g][v, p] = (4.0 * central(0.5 * h) - central(h)) / 3.0
                ncol += 1
    _say(case, "dense Jacobian columns", ncol)
    for g, gr in enumerate(orc.grids):
        act = gr.iblank.astype(bool)
        assert np.all(got[g][:, ~act] == 0.0), g
        for v in range(nv):
            a, b = got[g][v, act], want[g][v, act]
            tol = 1e-7 * np.maximum(np.abs(b), 1e-3 * np.max(np.abs(b)))
            err = np.abs(a - b)
            _say(case, "grid", g, "var", v, "max |err| / tol", float(np.max(err / tol)))
            assert np.all(err <= tol), (case, g, v, float(np.max(err / tol)))
