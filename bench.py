"""Benchmark: multi-rate vs single-rate Adams-Bashforth on the cylinder-like
overset workload, one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-equal-error] [--no-3d] [--tile-shapes S0,S1]

Workload (synthetic stand-in for the paper's cylinder case): a 512 x 512
Cartesian background on [-20, 20]^2 with far-field faces and a hole r < 2, and
a 256 x 128 body-fitted O-mesh (r = 0.5..3, stretching 1.03) with an
isothermal no-slip wall; Mach 0.2, Re 200, Pr 0.72, seeded 1e-3 perturbation
of u; SBP 4-2, cubic donors, fourth-order AB, rate ratio 4 (O-mesh 4 steps per
background step).

A step is one macrostep of the whole path (donor gather + per-grid fused
right-hand side, SAT and AB update for every evaluating grid).  The timed
region holds exactly K macrosteps with the states already in device memory.
value = MRAB point-updates per second = sum_l r_l * N_l(active) * K / time.

Also reported: the single-rate AB (every grid at the fast step) rate; the
equal-error comparison of both against a single-rate reference at a 32x
smaller step; the 3D three-level case (192^3 background, two 96^3 patches, a
64^3 patch; rates 1, 2, 2, 4), whose right-hand-side pass pair is the
HBM-bound kernel and gives the line's "roofline" (each launch timed with HIP
events on the stream it runs on, next to the kernel-trace durations and the
HBM traffic per launch of the committed profiles when they match the kernels'
source; the cylinder's fused kernel is "roofline_cylinder"); and the CPU oracle
on bounded samples of both workloads, on every host core and on one.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(rates=(1, 4)):
    import workloads
    wl = workloads.cylinder()
    wl.grids[0].rate, wl.grids[1].rate = rates
    return wl


TGV3D_WORKLOAD = ("3D periodic 192^3 + 2 x 96^3 (half spacing) + 64^3 (quarter spacing), SBP 4-2, cubic donors, "
                  "AB3, rates 1/2/2/4, Re 1600, M 0.3")


def tgv3d_measure(args):
    """The 3D three-level case (192^3 background, two 96^3 patches, one 64^3
    patch; rates 1, 2, 2, 4; SBP 4-2, AB3) -- the HBM-bound configuration:
    MRAB pt-updates/s over K macrosteps (per-grid streams, the library's
    plan at this size), then the roofline of the right-hand-side pass pair
    from a single-stream pass of K macrosteps with every launch between HIP
    events, next to the kernel-trace durations of the committed profile."""
    import torch
    import workloads
    from paper_1805_06607_amd.system import System
    wl = workloads.tgv3d()
    log("setup 3D system")
    s = System(wl)
    h, H = s.timestep()
    s.start(0.0)
    n_act = active_counts(s)
    pts = sum(g.rate * n for g, n in zip(wl.grids, n_act))
    s.macrostep(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.macrostep(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s.guard()
    log(f"3D MRAB {args.steps} macrosteps: {el * 1e3:.2f} ms")
    # launch durations from a single-stream pass (on the per-grid streams the
    # grids' launches overlap and each event pair would also time the others)
    s.set_option("multi_stream", 0)
    roof = timed_pass(s, wl, n_act, args.steps, "gradient pass (viscous stress and heat terms) + flux divergence, "
                                                "SAT and fused AB update on LDS tiles (k_grad_tile3d 16x8x8 + "
                                                "k_rhs_tile3d 16x8x4), all grids' launches of a macrostep")
    roof["workload"] = TGV3D_WORKLOAD
    s.close()
    return {"value": pts * args.steps / el, "unit": "pt-updates/s", "ms_per_step": el / args.steps * 1e3,
            "steps": args.steps, "points_active": n_act, "rates": [g.rate for g in wl.grids], "H": H,
            "roofline": roof, "_wl": wl}


def run_tgv3d(args):
    """Secondary mode: the 3D case alone.  Prints one JSON line of its own."""
    r = tgv3d_measure(args)
    wl = r.pop("_wl")
    line = {"metric": "MRAB pt-updates/s (3D three-level case), 1 GPU", "value": r["value"],
            "unit": "pt-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["ms_per_step"], "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": TGV3D_WORKLOAD, "points_active": r["points_active"], "H": r["H"]},
            "roofline": r["roofline"]}
    if not args.no_cpu:
        log("cpu baseline (3D)")
        line["cpu_baseline"] = cpu_baseline_3d(args, wl)
    print(json.dumps(line), flush=True)


def run_stability(args):
    """Stability mode: largest stable macrostep of single- and multi-rate AB
    (perturbation growth over 500 macrosteps from a steady state, GPU) on a
    cylinder-like stand-in without the wall (40^2 background, 96 x 24 O-mesh,
    uniform Mach 0.2 flow, a steady state of the discretisation), for AB3
    and AB34 and step ratios 1..8: r_SRAB = H_max(SR) / H_max(1) as in the
    paper's stability tables.  Prints one JSON line."""
    import workloads
    from paper_1805_06607_amd.system import System
    from paper_1805_06607_amd.stability import largest_stable_by_growth

    def wl_for(sr, order, m):
        return workloads.cylinder(nbg=40, ntheta=96, nr=24, half=6.0, rate_fast=sr, order=order, hist_len=m,
                                  wall=False, perturb=0.0)

    # fastest grid's own step estimate (eq. ts_overall with CFL 1, every grid at rate 1)
    w1 = wl_for(1, 3, 3)
    w1.params["cfl"] = 1.0
    s = System(w1)
    _, dt_fast = s.timestep()
    s.close()
    table = {}
    t0 = time.perf_counter()
    for order, m in ((3, 3), (3, 4)):
        name = f"AB{order}{m if m != order else ''}"
        rows = []
        for sr in (1, 2, 3, 4, 5, 6, 8):
            g = dt_fast * sr
            H = largest_stable_by_growth(lambda: System(wl_for(sr, order, m)), 0.1 * g, 4.0 * g, 0.005 * g)
            rows.append({"SR": sr, "H_max": H})
            log(f"{name} SR={sr} H_max={H:.6g}")
        for r in rows:
            r["r_SRAB"] = r["H_max"] / rows[0]["H_max"]
            r["efficiency"] = r["r_SRAB"] / r["SR"]
        table[name] = rows
    line = {"metric": "largest stable macrostep vs step ratio (MRAB stability), 1 GPU", "unit": "non-dimensional time",
            "value": table["AB34"][0]["H_max"], "higher_is_better": True, "n_gpus": 1, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "cylinder-like stand-in without wall: 40^2 background on [-6,6]^2 (hole r<2) + "
                                   "96x24 O-mesh (r 0.5..3), uniform flow M 0.2, Re 200, SBP 4-2, cubic donors",
                       "criterion": "growth of a 1e-8 random perturbation of the steady state over 500 "
                                    "macrosteps below 100 (eigenvalue modulus above ~1.009 flagged)",
                       "dt_fast_estimate": dt_fast},
            "table": table, "seconds": time.perf_counter() - t0}
    print(json.dumps(line), flush=True)


def run_batch(args):
    """Batch mode: 64 independent vortex systems of uneven size (background
    side U{64..512} at spacing 10/64, patch side U{S/4..S/2} at half spacing,
    seeded vortex positions, patch rate from {1, 2, 4}; SBP 2-1, bilinear,
    AB3), advanced together (one work-list launch per kind of job and
    micro-time) and, for comparison, one after another on their own.
    Prints one JSON line."""
    import torch
    import workloads
    from paper_1805_06607_amd.batch import Batch
    from paper_1805_06607_amd.system import System
    wls = workloads.batch_vortex(64, seed=3)
    log("setup 64 systems")
    systems = []
    for wl in wls:
        s = System(wl)
        s.timestep()
        s.start(0.0)
        systems.append(s)
    pts = sum(g.rate * int(ib.sum()) for s in systems for g, ib in zip(s.wl.grids, s.iblanks))
    npts = sum(g.npts for wl in wls for g in wl.grids)
    b = Batch(systems)
    best, tune_ms = b.autotune(reps=10)
    log(f"batch autotuner: shape {best}; ms per pass by shape (-1: each grid's own): "
        + ", ".join(f"{k}: {v:.3f}" for k, v in tune_ms.items()))
    b.macrostep(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.macrostep(args.steps)
    torch.cuda.synchronize()
    el_b = time.perf_counter() - t0
    log(f"batch: {args.steps} macrosteps {el_b * 1e3:.1f} ms")
    for s in systems:
        s.macrostep(args.warmup)
    torch.cuda.synchronize()
    ks = max(1, args.steps // 5)
    t0 = time.perf_counter()
    for _ in range(ks):
        for s in systems:
            s.macrostep(1)
    torch.cuda.synchronize()
    el_s = time.perf_counter() - t0
    bpp = 8 * 4 * (3 + 2)
    rl = batch_roofline(systems, best, tune_ms, bpp)
    line = {"metric": "batched MRAB pt-updates/s (64 uneven systems), 1 GPU", "value": pts * args.steps / el_b,
            "unit": "pt-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": el_b / args.steps * 1e3, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "64 vortex systems, background U{64..512}^2 + patch U{S/4..S/2}^2, rates "
                                   "{1,2,4}, SBP 2-1, bilinear, AB3, seed 3", "points": npts,
                       "point_updates_per_macrostep": pts},
            "tile_shape": best, "autotune_ms_per_rhs_pass_by_tile_shape": {str(k): v for k, v in tune_ms.items()},
            "one_system_at_a_time": {"value": pts * ks / el_s, "ms_per_step": el_s / ks * 1e3},
            "batch_speedup": (el_s / ks) / (el_b / args.steps),
            "algorithmic_GB_per_s": pts * bpp * args.steps / el_b / 1e9,
            "bytes_per_point": bpp, "roofline": rl}
    b.close()
    print(json.dumps(line), flush=True)


def batch_roofline(systems, shape, tune_ms, bpp):
    """Roofline of the batch's dominant launch, the one in which every grid of
    every system takes a fused right-hand side + AB update (all grids
    Cartesian, one tile shape: one work-list launch): algorithmic bytes
    (bpp x active points of every grid) / its duration, HIP-event timed by
    the batch autotuner on the batch's stream (reps passes after a warm-up
    pass).  Next to it the committed kernel-trace duration and counter
    traffic of that launch, when taken on the kernels as they are now."""
    from paper_1805_06607_amd.batch import tile_shape_info
    if shape < 0 or any(g.kind == 1 for s in systems for g in s.wl.grids):
        return None
    tx, ty, tm = tile_shape_info(shape)
    threads = sum(-(-g.n[0] // tx) * -(-g.n[1] // ty) * tx * ty * tm for s in systems for g in s.wl.grids)
    key = f"k_rhs_tiles<{int(systems[0].wl.params['sbp'])}, 1, {tx}, {ty}, {tm}> grid={threads}"
    n_act = sum(int(ib.sum()) for s in systems for ib in s.iblanks)
    bl = n_act * bpp
    avg = tune_ms[shape] * 1e-3
    ach = bl / avg / 1e9
    out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
           "traffic": stored_traffic().get(key), "kernel": key, "points": n_act, "bytes_per_point": bpp,
           "bytes_per_launch": bl, "avg_launch_us": avg * 1e6,
           "timing": "HIP events around the batch autotuner's timed passes on the batch's stream"}
    kt = stored_trace().get(key)
    if kt:
        out["kernel_trace_us"] = kt
        out["frac_kernel_trace"] = bl / (kt * 1e-6) / 1e9 / HBM_PEAK_GBS
        out["kernel_trace_source"] = "profiles/kernel_trace.txt"
    return out


def run_adjoint(args):
    """Adjoint mode: the cylinder case over --adj-macrosteps MRAB macrosteps
    (after the RK bootstrap).  J = time integral (trapezoid over the O-mesh's
    own steps) of the wall pressure force along x, sum over the wall points of
    p n_x r dtheta.  Its gradient with respect to the initial states -- the
    background's as a function of its u perturbation field (512 x 512 values)
    through torch autograd over the initial-condition map, the O-mesh's
    directly -- comes from the library's discrete adjoint (binomial
    checkpointing with --adj-snapshots snapshots).  Check: central
    differences with one Richardson step of the library's forward pass on 32
    seeded unit directions of (u perturbation, O-mesh state).  Over 200
    macrosteps (t = 200 H) no wave from the background reaches the wall
    (the O-mesh's outer boundary is 2.5 away), so J depends on the background
    perturbation only below rounding; the O-mesh state carries the
    sensitivity.  Prints one JSON line."""
    import torch
    import workloads
    from paper_1805_06607_amd.adjoint import Adjoint, MRABRun, schedule_cost, wall_objective
    from paper_1805_06607_amd.system import System
    nmacro, nsnap = args.adj_macrosteps, args.adj_snapshots
    wl = workloads.cylinder()
    s = System(wl)
    h, H = s.timestep()
    s.autotune(reps=10)
    adj = Adjoint(s, nsnap)
    pts, w = wall_objective(wl.grids[1])
    adj.set_objective(1, pts, w)
    dev = s.device
    gamma = wl.params["gamma"]
    q0 = torch.as_tensor(np.asarray(wl.q0[0], dtype=np.float64).reshape(4, -1), device=dev)
    q1 = torch.as_tensor(np.asarray(wl.q0[1], dtype=np.float64).reshape(4, -1), device=dev)
    p_inf = (gamma - 1.0) * (wl.params["q_inf"][3] - 0.5)      # uniform flow rho = 1, u = 1
    du0 = q0[1] / q0[0] - 1.0

    def ic(du):
        one = torch.ones_like(du)
        u = 1.0 + du
        return torch.stack([one, u, 0.0 * one, p_inf / (gamma - 1.0) + 0.5 * u * u])

    ic_err = float((ic(du0) - q0).abs().max())
    log(f"adjoint: initial-condition map reproduces the workload state to {ic_err:.2e}; H = {H:.4e}")
    adj.forward(nmacro, [ic(du0), q1])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J, _ = adj.forward(nmacro, [ic(du0), q1])
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    du = du0.clone().requires_grad_(True)
    qo = q1.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = MRABRun.apply(adj, nmacro, ic(du), qo)
    out[0].backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    gu, go = du.grad.detach(), qo.grad.detach()
    Jv = float(out[0].detach())
    log(f"adjoint: J = {Jv:.10e}, forward {t_fwd * 1e3:.1f} ms, gradient {t_grad * 1e3:.1f} ms "
        f"({adj.last_nfwd} forward macrosteps); |dJ/du| = {float(torch.linalg.vector_norm(gu)):.3e}, "
        f"|dJ/dq_omesh| = {float(torch.linalg.vector_norm(go)):.3e}")
    rng = np.random.default_rng(4)
    eps = args.adj_fd_eps
    rels, fds = [], []
    nu, no = du0.numel(), q1.numel()
    for k in range(32):
        v = rng.standard_normal(nu + no)
        v /= np.linalg.norm(v)
        vu = torch.as_tensor(v[:nu], device=dev)
        vo = torch.as_tensor(v[nu:].reshape(4, -1), device=dev)
        dd = float((gu * vu).sum() + (go * vo).sum())

        def f(e):
            return adj.forward(nmacro, [ic(du0 + e * vu), q1 + e * vo])[0]

        d1 = (f(eps) - f(-eps)) / (2.0 * eps)
        d2 = (f(0.5 * eps) - f(-0.5 * eps)) / eps
        fd = (4.0 * d2 - d1) / 3.0
        rels.append(abs(dd - fd) / max(abs(fd), 1e-300))
        fds.append(fd)
        log(f"  direction {k}: adjoint {dd:+.12e} fd {fd:+.12e} rel {rels[-1]:.2e}")
    # the background perturbation alone, seeded unit directions: central
    # differences see no change of J at this horizon
    fd_u = []
    for k in range(4):
        v = rng.standard_normal(nu)
        vu = torch.as_tensor(v / np.linalg.norm(v), device=dev)
        fd_u.append((adj.forward(nmacro, [ic(du0 + eps * vu), q1])[0]
                     - adj.forward(nmacro, [ic(du0 - eps * vu), q1])[0]) / (2.0 * eps))
    line = {"metric": "discrete-adjoint gradient of the time-integrated wall pressure force (cylinder, MRAB), 1 GPU",
            "value": t_grad, "unit": "s", "n_gpus": 1, "steps": nmacro, "warmup": 1,
            "ms_per_step": t_grad / nmacro * 1e3, "higher_is_better": False, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "cylinder-like overset: 512x512 background + 256x128 O-mesh, SBP 4-2, cubic "
                                   "donors, AB4 MRAB ratio 4; RK4 bootstrap then MRAB macrosteps; gradient with "
                                   "respect to the 512x512 initial u perturbation and the O-mesh initial state",
                       "macrosteps": nmacro, "snapshots": nsnap, "H": H},
            "J": Jv, "forward_s": t_fwd, "gradient_over_forward": t_grad / t_fwd,
            "forward_macrosteps_run": adj.last_nfwd,
            "schedule_recomputed_macrosteps": schedule_cost(nmacro, nsnap),
            "grad_norm_u_perturbation": float(torch.linalg.vector_norm(gu)),
            "grad_norm_omesh_state": float(torch.linalg.vector_norm(go)),
            "fd_check": {"directions": 32, "seed": 4, "eps": eps, "richardson": True,
                         "space": "unit vectors of (u perturbation 512x512, O-mesh state 4x256x128)",
                         "max_rel_err": max(rels), "median_rel_err": float(np.median(rels)),
                         "min_abs_fd": float(np.min(np.abs(fds)))},
            "fd_u_perturbation_only": fd_u,
            "workspace_bytes": adj.nbytes}
    print(json.dumps(line), flush=True)


TILE3D = (16, 8, 4)   # the 3D flux pass's default LDS tile (option rhs_tile3d = 1)
GRAD3D = (16, 8, 8)   # the 3D gradient pass's default LDS tile (option grad_tile3d = 4)


def kernel_names(sysg, wl):
    """Per grid: the key of its right-hand-side launches in the counter
    summary (the fused 2D kernel's instantiation, or for 3D the gradient +
    flux pass pair by its launch size in threads) and the kernel-trace keys
    (instantiation and launch size) of the launches one step makes."""
    names = []
    sbp = int(wl.params["sbp"])
    if wl.dim == 3:
        tile, gtile = "{}, {}, {}".format(*TILE3D), "{}, {}, {}".format(*GRAD3D)
        for gr in wl.grids:
            threads, gthreads = 1, 1
            for n, t, u in zip(gr.n, TILE3D, GRAD3D):
                threads *= -(-n // t) * t
                gthreads *= -(-n // u) * u
            names.append((f"tile3d_pair grid={threads}",
                          [f"k_grad_tile3d<{sbp}, {gtile}> grid={gthreads}",
                           f"k_rhs_tile3d<{sbp}, {tile}> grid={threads}"]))
        return names
    for g, gr in enumerate(wl.grids):
        shape, tx, ty, tm = sysg.tile_shape(g)
        if shape < 0:
            names.append((None, []))
            continue
        k = f"k_rhs_tile2d<{sbp}, {0 if gr.kind == 1 else 1}, {tx}, {ty}, {tm}>"
        threads = (-(-gr.n[0] // tx)) * (-(-gr.n[1] // ty)) * tx * ty * tm
        names.append((k, [f"{k} grid={threads}"]))
    return names


def stored_trace():
    """Average kernel durations [us] from the committed kernel-trace summary,
    keyed 'instantiation grid=threads', if it was taken on the kernels as they
    are now (same source hash)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "kernel_trace.txt")
    src = os.path.join(ROOT, "paper_1805_06607_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return {}
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    out, ok = {}, False
    with open(path) as f:
        for ln in f:
            ln = ln.strip()
            if ln.startswith("kernels_sha256"):
                ok = ln.split("=", 1)[1].strip() == sha
            elif ln.startswith("k_") and " avg_us=" in ln:
                key, val = ln.rsplit(" avg_us=", 1)
                out[key.strip()] = float(val)
    return out if ok else {}


def stored_traffic():
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the kernels as they are now (same source hash)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    src = os.path.join(ROOT, "paper_1805_06607_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return {}
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    out, ok = {}, False
    with open(path) as f:
        for ln in f:
            ln = ln.strip()
            if ln.startswith("kernels_sha256"):
                ok = ln.split("=", 1)[1].strip() == sha
            elif ln.startswith("k_") and "bytes_per_launch=" in ln:
                name, val = ln.rsplit("bytes_per_launch=", 1)
                out[name.strip()] = float(val)
                out.setdefault(name.split(" grid=")[0].strip(), float(val))
            elif ln.startswith("tile3d_pair") and "bytes_per_launch=" in ln:
                name, val = ln.rsplit("bytes_per_launch=", 1)
                out[name.strip()] = float(val)
    return out if ok else {}


def timed_pass(sysg, wl, n_act, steps, what):
    """K more macrosteps with every fused right-hand-side launch between HIP
    events on its stream; the roofline of those launches."""
    import torch
    sysg.kernel_timing(-2, steps * sum(g.rate for g in wl.grids))
    sysg.macrostep(steps)
    torch.cuda.synchronize()
    out = roofline(sysg, wl, n_act, what)
    sysg.kernel_timing(-1, 0)
    return out


def roofline(sysg, wl, n_act, what):
    """Roofline of the fused right-hand-side step over every timed launch of
    the timed region: algorithmic bytes (bytes_per_point x active points per
    launch) / summed launch duration, and per grid.  Next to the event-timed
    durations (which include each launch's dispatch latency): the kernel-trace
    durations of the committed profile, when it was taken on the kernels as
    they are now."""
    per_grid, tb, tt, tn = [], 0.0, 0.0, 0
    names = kernel_names(sysg, wl)
    traffic = stored_traffic()
    trace = stored_trace()
    tr_bytes, tr_ok = 0.0, True
    kt_time, kt_ok = 0.0, True
    for g in range(len(wl.grids)):
        ms, cnt = sysg.kernel_time(g)
        if cnt == 0:
            continue
        bpp = bytes_per_point(wl, g)
        bl = n_act[g] * bpp
        avg = ms * 1e-3 / cnt
        ach = bl / avg / 1e9
        key, launches = names[g]
        d = {"grid": g, "n": list(wl.grids[g].n), "kernel": key, "points": n_act[g], "bytes_per_point": bpp,
             "bytes_per_launch": bl, "launches": cnt, "avg_launch_us": avg * 1e6, "achieved": ach,
             "frac": ach / HBM_PEAK_GBS}
        if all(k in trace for k in launches):
            kt = sum(trace[k] for k in launches)
            d["kernel_trace_us"] = kt
            d["kernel_trace_launches"] = launches
            d["frac_kernel_trace"] = bl / (kt * 1e-6) / 1e9 / HBM_PEAK_GBS
            kt_time += kt * 1e-6 * cnt
        else:
            kt_ok = False
        if key in traffic:
            d["traffic"] = traffic[key]
            tr_bytes += traffic[key] * cnt
        else:
            tr_ok = False
        per_grid.append(d)
        tb += bl * cnt
        tt += ms * 1e-3
        tn += cnt
    ach = tb / tt / 1e9
    out = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
           "traffic": (tr_bytes / tn) if (tr_ok and tn) else None, "kernel": what,
           "bytes_per_launch": tb / tn, "avg_launch_us": tt / tn * 1e6, "launches_timed": tn,
           "timing": "HIP events around each launch on its stream (includes dispatch latency)"}
    if kt_ok and tn:
        out["kernel_trace_avg_launch_us"] = kt_time / tn * 1e6
        out["frac_kernel_trace"] = tb / kt_time / 1e9 / HBM_PEAK_GBS
        out["kernel_trace_source"] = "profiles/kernel_trace.txt"
    out["per_grid"] = per_grid
    return out


def active_counts(sysg):
    return [int(ib.sum()) for ib in sysg.iblanks]


def bytes_per_point(wl, g):
    """Algorithmic bytes per point of one fused right-hand-side + AB update:
    read the state, read m-1 older history values, write the new right-hand
    side, write the next state (nv doubles each), plus 5 metric doubles on
    curvilinear 2D grids."""
    nv = wl.dim + 2
    m = wl.params["hist_len"]
    b = 8 * nv * (m + 2)
    if wl.grids[g].kind == 1:
        b += 8 * (wl.dim * wl.dim + 1)
    return b


def run_gpu(args):
    import torch
    from paper_1805_06607_amd.system import System

    res = {}
    # ---------------------------------------------------------------- MRAB
    wl = workload((1, 4))
    log("setup MRAB system")
    mr = System(wl)
    h, H = mr.timestep()
    mr.start(0.0)
    if args.tile_shapes:
        # fixed shapes (counter runs: the profiler's own overhead would sway the autotuner)
        for g, sh in enumerate(int(x) for x in args.tile_shapes.split(",")):
            mr.set_tile_shape(g, sh)
        tiles = [mr.tile_shape(g) for g in range(mr.ngrids)]
    else:
        tiles = mr.autotune(reps=20)
    log(f"tile shapes (shape, tx, ty, threads per output): {tiles}")
    n_act = active_counts(mr)
    rates = [g.rate for g in wl.grids]
    pts_per_step = sum(r * n for r, n in zip(rates, n_act))
    mr.macrostep(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mr.macrostep(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt_mrab = t1 - t0
    mr.guard()
    log(f"MRAB {args.steps} macrosteps: {dt_mrab * 1e3:.2f} ms")
    res["mrab"] = dict(time_s=dt_mrab, pts_per_step=pts_per_step, H=H, h=h, tiles=tiles)
    # roofline of the dominant kernel: the fused right-hand-side step, every
    # launch (1 background + 4 O-mesh per macrostep) of a second pass of K
    # macrosteps identical to the timed one, each launch between HIP events
    # (the events themselves cost host time, so the throughput above is taken
    # without them)
    res["roofline_cylinder"] = timed_pass(mr, wl, n_act, args.steps,
                                          "k_rhs_tile2d (fused gradients, flux divergence, SAT, AB update), "
                                          "all launches of a macrostep (background and O-mesh)")
    del mr
    # ---------------------------------------------------------------- SRAB
    wls = workload((1, 1))
    wls.params["dt_fixed"] = h            # every grid at the fast step
    log("setup SRAB system")
    sr = System(wls)
    sr.timestep()
    sr.start(0.0)
    sr.autotune(reps=20)
    sr.macrostep(args.warmup)
    torch.cuda.synchronize()
    nsr = args.steps * 4
    t0 = time.perf_counter()
    sr.macrostep(nsr)
    torch.cuda.synchronize()
    dt_srab = time.perf_counter() - t0
    srab_pts = sum(n_act) * nsr
    log(f"SRAB {nsr} steps: {dt_srab * 1e3:.2f} ms")
    res["srab"] = dict(time_s=dt_srab, steps=nsr, pts=srab_pts)
    del sr
    # -------------------------------------------------------- equal error
    if not args.no_equal_error:
        res["equal_error"] = equal_error(args, h)
    # ------------------------------------ 3D case: the HBM roofline config
    if not args.no_3d:
        res["tgv3d"] = tgv3d_measure(args3d(args))
        res["roofline"] = res["tgv3d"]["roofline"]
    else:
        res["roofline"] = res["roofline_cylinder"]
    return res, wl, n_act


def args3d(args):
    """The 3D part of the default run: K = max(5, steps / 20) macrosteps
    (a 3D macrostep is ~30x a cylinder macrostep), 2 warm-up macrosteps."""
    a = argparse.Namespace(**vars(args))
    a.steps = max(5, args.steps // 20)
    a.warmup = 2
    return a


def equal_error(args, h):
    """MRAB (macrostep 4 hh, O-mesh at hh) for hh in {h, h/2, h/4} and
    single-rate AB (every grid at hh) for hh in {h, h/2, h/4, h/8}, against a
    single-rate reference at h/32, all from the same initial state and
    stopped at the same final time T = 4h (m - 1 + N) (each bootstrap spans
    m - 1 of its own macrosteps); error = max |rho - rho_ref| over active
    points of both grids (the paper's error measure for its convergence
    tables).  Wall time covers the macrosteps only.  Single-rate AB cannot
    step above h (the O-mesh's stable step), so its curve starts at h.
    Reported: single-rate wall time at each MRAB error (log-log interpolation
    inside the single-rate points; MRAB's errors lie inside their range) over
    MRAB's wall time, and single-rate error at each MRAB wall time where that
    wall time lies inside the single-rate range (None elsewhere: no
    clamping)."""
    import torch
    from paper_1805_06607_amd.system import System
    N = args.ee_macrosteps
    wl0 = workload((1, 4))
    m = wl0.params["hist_len"]

    # common start: the impulsive start (uniform flow meeting a no-slip wall) is
    # first developed by a single-rate run at h/4, so that the bootstraps of
    # the compared runs see a smooth solution
    spin = workload((1, 1))
    spin.params["dt_fixed"] = h / 4
    s = System(spin)
    s.timestep()
    s.start(0.0)
    s.macrostep(args.ee_spinup)
    q_start = [s.state(g).cpu().numpy() for g in range(2)]
    del s

    def run(rates, H, nsteps):
        wl = workload(rates)
        wl.q0 = [q.copy() for q in q_start]
        wl.params["dt_fixed"] = H
        s = System(wl)
        s.timestep()
        s.autotune(reps=10)
        s.start(0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.macrostep(nsteps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        t, _ = s.time()
        rho = [s.state(g)[0].cpu().numpy() for g in range(2)]
        ib = [x.astype(bool) for x in s.iblanks]
        del s
        return rho, ib, el, t

    # reference: every grid at h/32, T = 4h (m - 1 + N) = (h/32)(m - 1 + n)
    ref, ib, el_ref, t_ref = run((1, 1), h / 32, 128 * (m - 1 + N) - (m - 1))

    def err(rho):
        return max(float(np.max(np.abs(rho[g] - ref[g])[ib[g]])) for g in range(2))

    mrab, srab = [], []
    for f in (1, 2, 4):
        hh = h / f
        Nh = f * (N + m - 1) - (m - 1)
        rho_m, _, el_m, t_m = run((1, 4), 4 * hh, Nh)
        mrab.append({"h": hh, "macrosteps": Nh, "err": err(rho_m), "wall_s": el_m, "T": t_m})
        log(f"equal error MRAB h/{f}: err {mrab[-1]['err']:.3e} wall {el_m:.4f}s")
    for f in (1, 2, 4, 8):
        hh = h / f
        ns = 4 * f * (N + m - 1) - (m - 1)
        rho_s, _, el_s, t_s = run((1, 1), hh, ns)
        srab.append({"h": hh, "steps": ns, "err": err(rho_s), "wall_s": el_s, "T": t_s})
        log(f"equal error SRAB h/{f}: err {srab[-1]['err']:.3e} wall {el_s:.4f}s")
    lw = np.log([p["wall_s"] for p in srab])
    le = np.log([p["err"] for p in srab])
    ow, oe = np.argsort(lw), np.argsort(le)
    wall_ratio, err_ratio = [], []
    for p in mrab:
        x = np.log(p["err"])
        if le[oe][0] <= x <= le[oe][-1]:
            w_s = float(np.exp(np.interp(x, le[oe], lw[oe])))
            wall_ratio.append(w_s / p["wall_s"])
        else:
            wall_ratio.append(None)
        x = np.log(p["wall_s"])
        if lw[ow][0] <= x <= lw[ow][-1]:
            e_s = float(np.exp(np.interp(x, lw[ow], le[ow])))
            err_ratio.append(e_s / p["err"])
        else:
            err_ratio.append(None)
    log(f"equal error: T={t_ref:.6g}; single-rate wall time at MRAB's error / MRAB wall time = "
        + ", ".join("-" if r is None else f"{r:.2f}" for r in wall_ratio))
    first_m, first_s = mrab[0], srab[0]
    return {"T": t_ref, "mrab_macrosteps": N, "spinup_steps_at_h_over_4": args.ee_spinup,
            "err_mrab": first_m["err"], "err_srab": first_s["err"],
            "wall_s_mrab": first_m["wall_s"], "wall_s_srab": first_s["wall_s"],
            "wall_ratio_srab_over_mrab_same_h": first_s["wall_s"] / first_m["wall_s"],
            "mrab": mrab, "srab": srab,
            "srab_wall_at_mrab_err_over_mrab_wall": wall_ratio,
            "srab_err_at_mrab_wall_over_mrab_err": err_ratio,
            "mrab_faster_at_equal_error": bool(all(r is not None and r > 1.0 for r in wall_ratio)),
            "reference": "single-rate AB at h/32", "error": "max |rho - rho_ref| over active points"}


def _omp():
    """The OpenMP runtime the oracle's C part runs on (thread count control)."""
    import ctypes
    lib = ctypes.CDLL("libgomp.so.1")
    lib.omp_get_max_threads.restype = ctypes.c_int
    return lib


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _timed_macrosteps(mr, seconds, min_steps=1):
    t0 = time.perf_counter()
    k = 0
    while True:
        mr.macrostep()
        k += 1
        if time.perf_counter() - t0 > seconds and k >= min_steps:
            break
    return k, time.perf_counter() - t0


def cpu_baseline(args):
    """The oracle (plain C + numpy, OpenMP) on a bounded sample of the same
    workload: MRAB macrosteps from a history of repeated F(y0), timed until
    ~10 s of work on every core of the host, then for ~5 s on one core."""
    import oracle
    wl = workload((1, 4))
    orc = oracle.OracleSystem(wl)
    h, H = orc.timestep()
    mr = orc.integrator(H)
    F0 = orc.rhs(wl.q0)
    m = wl.params["hist_len"]
    mr.set_history(wl.q0, [[F0[g]] * m for g in range(2)], 0.0)
    n_act = [int(g.iblank.sum()) for g in orc.grids]
    pts = sum(g.rate * n for g, n in zip(wl.grids, n_act))
    omp = _omp()
    threads = omp.omp_get_max_threads()
    k, el = _timed_macrosteps(mr, args.cpu_seconds, 2)
    omp.omp_set_num_threads(1)
    k1, el1 = _timed_macrosteps(mr, args.cpu_seconds / 2)
    omp.omp_set_num_threads(threads)
    return {"value": pts * k / el, "unit": "pt-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} MRAB macrosteps of the same cylinder workload (full size) from a "
                      f"constant history, {el:.1f} s",
            "one_core": {"value": pts * k1 / el1, "cores": 1, "sample": f"{k1} more macrosteps, {el1:.1f} s"},
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}


def cpu_baseline_3d(args, wl=None):
    """The oracle on a bounded sample of the 3D three-level workload: one
    MRAB macrostep (all grids at their rates) from a history of repeated
    F(y0) on every core, and the right-hand side of the 64^3 inner patch on
    one core."""
    import oracle
    import workloads
    wl = wl if wl is not None else workloads.tgv3d()
    t0 = time.perf_counter()
    orc = oracle.OracleSystem(wl)
    setup = time.perf_counter() - t0
    h, H = orc.timestep()
    mr = orc.integrator(H)
    F0 = orc.rhs(wl.q0)
    m = wl.params["hist_len"]
    mr.set_history(wl.q0, [[F0[g]] * m for g in range(len(wl.grids))], 0.0)
    n_act = [int(g.iblank.sum()) for g in orc.grids]
    pts = sum(g.rate * n for g, n in zip(wl.grids, n_act))
    omp = _omp()
    threads = omp.omp_get_max_threads()
    k, el = _timed_macrosteps(mr, 0.0)
    omp.omp_set_num_threads(1)
    gi = len(wl.grids) - 1
    recv = orc.receiver_data(gi, wl.q0)
    t0 = time.perf_counter()
    orc.rhs_grid(gi, wl.q0[gi], recv)
    el1 = time.perf_counter() - t0
    omp.omp_set_num_threads(threads)
    return {"value": pts * k / el, "unit": "pt-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} MRAB macrostep of the 3D three-level workload (full size) from a constant history, "
                      f"{el:.1f} s (oracle setup {setup:.0f} s not counted)",
            "one_core": {"value": n_act[gi] / el1, "cores": 1,
                         "sample": f"one right-hand side of the {'x'.join(map(str, wl.grids[gi].n))} inner patch "
                                   f"({n_act[gi]} points), {el1:.1f} s"},
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-equal-error", action="store_true")
    ap.add_argument("--no-3d", action="store_true", help="leave out the 3D roofline part of the default run")
    ap.add_argument("--ee-macrosteps", type=int, default=200)
    ap.add_argument("--ee-spinup", type=int, default=2000)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--workload", default="cylinder", choices=["cylinder", "tgv3d", "stability", "batch", "adjoint"])
    ap.add_argument("--adj-macrosteps", type=int, default=200)
    ap.add_argument("--adj-snapshots", type=int, default=20)
    ap.add_argument("--adj-fd-eps", type=float, default=1e-3)
    ap.add_argument("--tile-shapes", default="",
                    help="comma-separated tile shape per grid of the cylinder case instead of the autotuner's")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the method's work here has no multi-GPU path "
              "(see the sharding design notes); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {args.calibrate_copy_mib} MiB read + {args.calibrate_copy_mib} MiB written")
        del a, c
    if args.workload == "tgv3d":
        run_tgv3d(args)
        return
    if args.workload == "stability":
        run_stability(args)
        return
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "adjoint":
        run_adjoint(args)
        return
    res, wl, n_act = run_gpu(args)
    K = args.steps
    t = res["mrab"]["time_s"]
    value = res["mrab"]["pts_per_step"] * K / t
    line = {
        "metric": "MRAB pt-updates/s & HBM roofline frac vs single-rate AB at equal error, 1 GPU",
        "value": value,
        "unit": "pt-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": t / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "cylinder-like overset: 512x512 Cartesian background (far field, hole r<2) + "
                        "256x128 O-mesh (wall), SBP 4-2, cubic donors, AB4 MRAB ratio 4, Re 200, M 0.2",
            "points_active": n_act, "rates": [g.rate for g in wl.grids],
            "H": res["mrab"]["H"], "h": res["mrab"]["h"], "tile_shapes": res["mrab"]["tiles"],
        },
        "roofline": res["roofline"],
        "roofline_cylinder": res["roofline_cylinder"],
        "srab": {
            "value": res["srab"]["pts"] / res["srab"]["time_s"],
            "ms_per_macrostep_equivalent": res["srab"]["time_s"] / res["srab"]["steps"] * 4 * 1e3,
            "mrab_speedup_same_fast_step": (res["srab"]["time_s"] / (res["srab"]["steps"] / 4)) / (t / K),
        },
        "equivalent_single_rate_pt_updates_per_s": max(g.rate for g in wl.grids) * sum(n_act) * K / t,
    }
    if "equal_error" in res:
        line["equal_error"] = res["equal_error"]
    if "tgv3d" in res:
        line["tgv3d"] = {k: v for k, v in res["tgv3d"].items() if k not in ("roofline", "_wl")}
        line["tgv3d"]["workload"] = TGV3D_WORKLOAD
    if not args.no_cpu:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(args)
        if "tgv3d" in res:
            log("cpu baseline (3D)")
            line["cpu_baseline_3d"] = cpu_baseline_3d(args, res["tgv3d"]["_wl"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
