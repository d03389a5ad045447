"""Seeded synthetic problem descriptions (inputs only).

This module describes *problems*: grid geometry, boundary-condition flags, hole
shapes, rate per grid, physical constants, scheme choices and initial states.
It holds none of the method's arithmetic (no SBP operators, metrics, fluxes,
penalties, interpolation weights or time-integration coefficients).  Both the
GPU product path and the independent CPU oracle build their own discretisation
from these descriptions.

Geometry conventions
--------------------
* Points are numbered x fastest: flat index ``p = i + nx*(j + ny*k)``.
* A Cartesian grid has ``x_d(i_d) = origin[d] + i_d*spacing[d]``.
* A curvilinear grid carries explicit coordinates ``coords`` of shape
  ``(dim, N)``, sampled at the integer indices of its continuous mapping
  ``mapping(F)`` (fractional indices ``F`` of shape ``(dim, K)`` to physical
  points), and the closed-form inverse of that mapping, ``inverse(X)``
  (physical points to fractional indices).  Both describe the grid's geometry;
  which of them a consumer uses to locate donor cells is its own choice.
* Holes are shapes; a point strictly inside any of its grid's shapes is blanked.

The problems follow the paper's workloads: the convecting isentropic vortex
(Appendix, "Spatial Accuracy of Solutions"), the cylinder in cross flow
(section "Guiding Experiment"), manufactured right-hand sides (Appendix,
"Spatial Accuracy of Right-Hand Sides"), plus a 3D three-level stand-in for the
large multi-grid jet case.  No dataset is used; every field is synthetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

# boundary-condition flags per grid face (order: -x, +x, -y, +y, -z, +z)
BC_PERIODIC = 0
BC_INTERFACE = 1
BC_FARFIELD = 2
BC_WALL = 3

CARTESIAN = 0
CURVILINEAR = 1


@dataclass
class Grid:
    name: str
    n: tuple                      # points per direction, x first
    periodic: tuple               # bool per direction
    kind: int                     # CARTESIAN | CURVILINEAR
    face_bc: list                 # 2*dim flags
    rate: int                     # right-hand-side evaluations per macrostep
    priority: int                 # donor preference: higher is finer
    origin: tuple = (0.0, 0.0, 0.0)
    spacing: tuple = (1.0, 1.0, 1.0)
    coords: Optional[np.ndarray] = None     # (dim, N) for curvilinear grids
    inverse: Optional[Callable] = None      # X (dim,K) -> fractional index (dim,K)
    mapping: Optional[Callable] = None      # fractional index (dim,K) -> X (dim,K)
    holes: list = field(default_factory=list)   # ('box', lo, hi) | ('disk', c, r)
    # coordinate jump across the seam of each periodic direction (curvilinear
    # grids on a translation-periodic domain): x(i_d + n_d) = x(i_d) + coord_period[d]
    coord_period: Optional[list] = None

    @property
    def dim(self):
        return len(self.n)

    @property
    def npts(self):
        return int(np.prod(self.n))

    def points(self) -> np.ndarray:
        """Physical coordinates, shape (dim, N), x fastest."""
        if self.kind == CURVILINEAR:
            return self.coords
        axes = [self.origin[d] + self.spacing[d] * np.arange(self.n[d]) for d in range(self.dim)]
        mesh = np.meshgrid(*axes[::-1], indexing="ij")[::-1]
        return np.stack([m.ravel() for m in mesh])

    def cartesian_inverse(self, X: np.ndarray) -> np.ndarray:
        o = np.asarray(self.origin[: self.dim])[:, None]
        h = np.asarray(self.spacing[: self.dim])[:, None]
        return (X - o) / h

    def frac_index(self, X: np.ndarray) -> np.ndarray:
        if self.kind == CARTESIAN:
            return self.cartesian_inverse(X)
        return self.inverse(X)


@dataclass
class Workload:
    name: str
    dim: int
    params: dict
    grids: List[Grid]
    q0: List[np.ndarray]          # per grid, (nv, N)
    macrosteps: int = 100
    notes: str = ""

    @property
    def nv(self):
        return self.dim + 2


def default_params(**kw) -> dict:
    p = dict(
        gamma=1.4, Re=1000.0, Pr=0.72, mu=1.0, lambda_over_mu=-2.0 / 3.0,
        sigma_I_iface=0.5, sigma_I_bc=1.0, T_wall=1.0, wall_visc=1.0,
        q_inf=[1.0, 0.0, 0.0, 0.0, 0.0],
        sbp=21, order=3, hist_len=3, interp_width=2,
        cfl=0.5, dt_fixed=0.0,
    )
    p.update(kw)
    return p


def conserved_from_primitive(rho, vel: Sequence[np.ndarray], p, gamma):
    """Pack (rho, rho*u_i, rho*E) with rho*E = p/(gamma-1) + rho*|u|^2/2."""
    ke = 0.5 * rho * sum(v * v for v in vel)
    return np.stack([rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke])


# ----------------------------------------------------------------------------
# isentropic vortex (exact Euler solution)
# ----------------------------------------------------------------------------
def vortex_state(x, y, t, gamma, omega, phi, x0, y0, u0, v0):
    """Convecting isentropic vortex with p_inf = rho_inf = 1 (c0^2 = gamma)."""
    c0sq = gamma
    dx = x - x0 - u0 * t
    dy = y - y0 - v0 * t
    r2 = dx * dx + dy * dy
    e = np.exp(1.0 - phi * phi * r2)
    rho = (1.0 - omega * omega * (gamma - 1.0) / (8.0 * math.pi ** 2 * c0sq) * e) ** (1.0 / (gamma - 1.0))
    es = np.exp(0.5 * (1.0 - phi * phi * r2))
    u = u0 - omega / (2.0 * math.pi) * phi * dy * es
    v = v0 + omega / (2.0 * math.pi) * phi * dx * es
    p = rho ** gamma
    return rho, u, v, p


def vortex_box(nbg: int = 64, npatch: int = 32, Re: float = 1000.0, rate_bg: int = 1,
               rate_patch: int = 2, order: int = 3, spacing: Optional[float] = None,
               centre: Optional[Sequence[float]] = None) -> Workload:
    """Periodic 64^2 background on [0,10)^2 with a 32^2 patch at half spacing.

    The patch is centred on an isentropic vortex (strength 5, advected at
    Mach 0.5).  SBP 2-1, bilinear donors, third-order MRAB with ratio 2.
    spacing (default 10 / nbg) sets the background spacing, so the periodic
    domain is nbg * spacing wide; centre (default the domain centre) places
    the vortex and the patch.
    """
    gamma = 1.4
    h = 10.0 / nbg if spacing is None else spacing
    L = nbg * h
    hp = h / 2.0
    cx, cy = (0.5 * L, 0.5 * L) if centre is None else centre
    c = cx
    half_patch = 0.5 * (npatch - 1) * hp
    g0 = Grid("background", (nbg, nbg), (True, True), CARTESIAN,
              [BC_PERIODIC] * 4, rate_bg, 0, origin=(0.0, 0.0, 0.0), spacing=(h, h, h))
    # hole: the patch box shrunk by four patch cells
    hh = half_patch - 4.0 * hp
    g0.holes.append(("box", (cx - hh, cy - hh), (cx + hh, cy + hh)))
    g1 = Grid("patch", (npatch, npatch), (False, False), CARTESIAN,
              [BC_INTERFACE] * 4, rate_patch, 1,
              origin=(cx - half_patch, cy - half_patch, 0.0), spacing=(hp, hp, hp))
    params = default_params(gamma=gamma, Re=Re, sbp=21, order=order, hist_len=order,
                            interp_width=2, cfl=0.5)
    u0 = 0.5 * math.sqrt(gamma)
    params["q_inf"] = [1.0, u0, 0.0, 1.0 / (gamma - 1.0) + 0.5 * u0 * u0, 0.0]
    params["T_wall"] = 1.0
    q0 = []
    for g in (g0, g1):
        X = g.points()
        rho, u, v, p = vortex_state(X[0], X[1], 0.0, gamma, 5.0, 1.0, cx, cy, u0, 0.0)
        q0.append(conserved_from_primitive(rho, [u, v], p, gamma))
    return Workload("vortex_box", 2, params, [g0, g1], q0, macrosteps=100,
                    notes="isentropic vortex box-in-box, SBP 2-1, bilinear, AB3 ratio 2")


def batch_vortex(nsys: int = 64, seed: int = 3, smin: int = 64, smax: int = 512,
                 spacing: float = 10.0 / 64.0, rates: Sequence[int] = (1, 2, 4)) -> List[Workload]:
    """Independent vortex systems of uneven size: background side
    S ~ U{smin..smax} at a common spacing, patch side ~ U{ceil(S/4)..floor(S/2)}
    at half spacing centred on a seeded vortex position (kept clear of the
    periodic seam), patch rate drawn from `rates`; AB3."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(nsys):
        S = int(rng.integers(smin, smax + 1))
        P = int(rng.integers(-(-S // 4), S // 2 + 1))
        r = int(rng.choice(np.asarray(rates)))
        L = S * spacing
        half = 0.5 * (P - 1) * spacing / 2.0
        lo, hi = half + 2.0 * spacing, L - half - 2.0 * spacing
        cx, cy = (float(rng.uniform(lo, hi)), float(rng.uniform(lo, hi)))
        out.append(vortex_box(nbg=S, npatch=P, rate_patch=r, spacing=spacing, centre=(cx, cy)))
    return out


# ----------------------------------------------------------------------------
# cylinder-like overset: Cartesian background + body-fitted O-mesh
# ----------------------------------------------------------------------------
def omesh_radii(nr: int, r0: float = 0.5, r1: float = 3.0, stretch: float = 1.03) -> np.ndarray:
    dr0 = (r1 - r0) * (stretch - 1.0) / (stretch ** (nr - 1) - 1.0)
    j = np.arange(nr, dtype=np.float64)
    return r0 + dr0 * (stretch ** j - 1.0) / (stretch - 1.0)


def omesh_grid(ntheta: int, nr: int, rate: int, priority: int, wall: bool = True,
               r0: float = 0.5, r1: float = 3.0, stretch: float = 1.03,
               outer_bc: int = BC_INTERFACE) -> Grid:
    r = omesh_radii(nr, r0, r1, stretch)
    th = 2.0 * math.pi * np.arange(ntheta) / ntheta
    R, TH = np.meshgrid(r, th, indexing="ij")          # (nr, ntheta): theta fastest
    coords = np.stack([(R * np.cos(TH)).ravel(), (R * np.sin(TH)).ravel()])
    dr0 = (r1 - r0) * (stretch - 1.0) / (stretch ** (nr - 1) - 1.0)

    def mapping(F, ntheta=ntheta, dr0=dr0):
        # theta = 2 pi i / ntheta, r = r0 + dr0 (stretch^j - 1) / (stretch - 1)
        F = np.asarray(F, dtype=np.float64)
        tt = 2.0 * math.pi * F[0] / ntheta
        rr = r0 + dr0 * (stretch ** F[1] - 1.0) / (stretch - 1.0)
        return np.stack([rr * np.cos(tt), rr * np.sin(tt)])

    def inverse(X, ntheta=ntheta, dr0=dr0):
        rr = np.hypot(X[0], X[1])
        tt = np.mod(np.arctan2(X[1], X[0]), 2.0 * math.pi)
        fi = tt / (2.0 * math.pi / ntheta)
        with np.errstate(invalid="ignore", divide="ignore"):
            fj = np.log1p((stretch - 1.0) * (rr - r0) / dr0) / math.log(stretch)
        return np.stack([fi, fj])

    bc_lo = BC_WALL if wall else BC_FARFIELD
    return Grid("omesh", (ntheta, nr), (True, False), CURVILINEAR,
                [BC_PERIODIC, BC_PERIODIC, bc_lo, outer_bc], rate, priority,
                coords=coords, inverse=inverse, mapping=mapping)


def cylinder(nbg: int = 512, ntheta: int = 256, nr: int = 128, half: float = 20.0,
             seed: int = 1, rate_fast: int = 4, order: int = 4, hist_len: Optional[int] = None,
             mach: float = 0.2, Re: float = 200.0, hole_r: float = 2.0, wall: bool = True,
             perturb: float = 1e-3) -> Workload:
    """Cylinder-like overset case: Cartesian background on [-half, half]^2
    (far-field faces) with a hole r < hole_r, and a 2D annular O-mesh
    (periodic in theta, geometric stretching 1.03 from r=0.5 to r=3) carrying an
    isothermal no-slip wall at r = 0.5.  Uniform flow at Mach 0.2 plus a seeded
    U(-perturb, perturb) perturbation of u on every background point.  With
    wall=False the inner face is far field too, and with perturb=0 the uniform
    flow is then a steady state of the discretisation (a base state for step
    matrices).
    """
    gamma = 1.4
    h = 2.0 * half / (nbg - 1)
    g0 = Grid("background", (nbg, nbg), (False, False), CARTESIAN,
              [BC_FARFIELD] * 4, 1, 0, origin=(-half, -half, 0.0), spacing=(h, h, h))
    g0.holes.append(("disk", (0.0, 0.0), hole_r))
    g1 = omesh_grid(ntheta, nr, rate_fast, 1, wall=wall)
    p_inf = 1.0 / (gamma * mach * mach)
    params = default_params(gamma=gamma, Re=Re, Pr=0.72, sbp=42, order=order,
                            hist_len=hist_len or order, interp_width=4, cfl=0.25)
    params["q_inf"] = [1.0, 1.0, 0.0, p_inf / (gamma - 1.0) + 0.5, 0.0]
    params["T_wall"] = p_inf / 1.0
    rng = np.random.Generator(np.random.PCG64(seed))
    du = rng.uniform(-perturb, perturb, size=g0.npts) if perturb > 0 else np.zeros(g0.npts)
    q0 = []
    for g, pert in ((g0, du), (g1, 0.0)):
        one = np.ones(g.npts)
        q0.append(conserved_from_primitive(one, [one * (1.0 + pert), 0.0 * one], p_inf * one, gamma))
    return Workload("cylinder", 2, params, [g0, g1], q0, macrosteps=1000,
                    notes="Cartesian background + O-mesh, SBP 4-2, cubic donors, AB4 ratio 4")


# ----------------------------------------------------------------------------
# 3D three-level case (Taylor-Green-like field, seeded phases)
# ----------------------------------------------------------------------------
def tgv3d(nbg: int = 192, npatch: int = 96, ninner: int = 64, seed: int = 2,
          order: int = 3, Re: float = 1600.0, mach: float = 0.3) -> Workload:
    """Periodic background on [0, 2pi)^3, two patches at half spacing centred at
    (pi/2, pi, pi) and (3pi/2, pi, pi), and an inner patch at quarter spacing
    inside the first patch (rates 1, 2, 2, 4).  Holes are the finer boxes
    shrunk by six finer cells.
    """
    gamma = 1.4
    L = 2.0 * math.pi
    h = L / nbg
    grids = []
    g0 = Grid("background", (nbg,) * 3, (True,) * 3, CARTESIAN, [BC_PERIODIC] * 6, 1, 0,
              origin=(0.0, 0.0, 0.0), spacing=(h, h, h))
    grids.append(g0)
    centres = [(math.pi / 2, math.pi, math.pi), (3 * math.pi / 2, math.pi, math.pi)]
    patches = []
    for idx, cen in enumerate(centres):
        hp = h / 2.0
        half_ext = 0.5 * (npatch - 1) * hp
        g = Grid(f"patch{idx + 1}", (npatch,) * 3, (False,) * 3, CARTESIAN, [BC_INTERFACE] * 6,
                 2, 1, origin=tuple(c - half_ext for c in cen), spacing=(hp, hp, hp))
        shrink = half_ext - 6.0 * hp
        g0.holes.append(("box", tuple(c - shrink for c in cen), tuple(c + shrink for c in cen)))
        patches.append(g)
        grids.append(g)
    hi = h / 4.0
    half_in = 0.5 * (ninner - 1) * hi
    cen = centres[0]
    g3 = Grid("inner", (ninner,) * 3, (False,) * 3, CARTESIAN, [BC_INTERFACE] * 6, 4, 2,
              origin=tuple(c - half_in for c in cen), spacing=(hi, hi, hi))
    shrink = half_in - 6.0 * hi
    patches[0].holes.append(("box", tuple(c - shrink for c in cen), tuple(c + shrink for c in cen)))
    grids.append(g3)
    p0 = 1.0 / (gamma * mach * mach)
    params = default_params(gamma=gamma, Re=Re, Pr=0.72, sbp=42, order=order, hist_len=order,
                            interp_width=4, cfl=0.4)
    params["q_inf"] = [1.0, 0.0, 0.0, 0.0, p0 / (gamma - 1.0)]
    params["T_wall"] = p0
    rng = np.random.Generator(np.random.PCG64(seed))
    ph = rng.uniform(0.0, 2.0 * math.pi, size=3)
    q0 = []
    for g in grids:
        X = g.points()
        x, y, z = X[0] + ph[0], X[1] + ph[1], X[2] + ph[2]
        u = np.sin(x) * np.cos(y) * np.cos(z)
        v = -np.cos(x) * np.sin(y) * np.cos(z)
        w = 0.0 * x
        rho = np.ones_like(x)
        p = p0 + (rho / 16.0) * (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0)
        q0.append(conserved_from_primitive(rho, [u, v, w], p, gamma))
    return Workload("tgv3d", 3, params, grids, q0, macrosteps=200,
                    notes="3D periodic background + 2 half-spacing patches + quarter-spacing patch")


# ----------------------------------------------------------------------------
# manufactured right-hand sides and other pins
# ----------------------------------------------------------------------------
def mms_box(N: int, viscous: bool, sbp: int = 42) -> Workload:
    """Box-in-box manufactured state: periodic [-1,1)^2 background with N^2
    points and a [-0.5,0.5]^2 patch at the same spacing.  Inviscid state
    rho*u = sin(2 pi (x-1/2)); viscous state rho*u = sin(2 pi (y-1/2)), with
    rho = 1, v = 0, p = 1 (so T is constant)."""
    gamma = 1.4
    h = 2.0 / N
    npatch = N // 2 + 1
    width = 4 if sbp == 42 else 2
    margin = 6 if width == 4 else 4
    g0 = Grid("outer", (N, N), (True, True), CARTESIAN, [BC_PERIODIC] * 4, 1, 0,
              origin=(-1.0, -1.0, 0.0), spacing=(h, h, h))
    hh = 0.5 - margin * h
    g0.holes.append(("box", (-hh, -hh), (hh, hh)))
    g1 = Grid("inner", (npatch, npatch), (False, False), CARTESIAN, [BC_INTERFACE] * 4, 1, 1,
              origin=(-0.5, -0.5, 0.0), spacing=(h, h, h))
    params = default_params(gamma=gamma, Re=(1.0 if viscous else math.inf), sbp=sbp,
                            order=3, hist_len=3, interp_width=width)
    params["q_inf"] = [1.0, 0.0, 0.0, 1.0 / (gamma - 1.0), 0.0]
    q0 = []
    for g in (g0, g1):
        X = g.points()
        s = np.sin(2 * math.pi * ((X[1] if viscous else X[0]) - 0.5))
        one = np.ones(g.npts)
        q0.append(conserved_from_primitive(one, [s, 0.0 * one], one, gamma))
    return Workload("mms_box", 2, params, [g0, g1], q0)


def vortex_convergence(N: int, sbp: int = 42) -> Workload:
    """Inviscid vortex (phi = 10, u0 = 2) on a periodic [-1,1) x [-1/2,1/2)
    background with an N x N patch on [-0.38, 0.38]^2; background spacing
    2/(2N) in x and 1/N in y so both grids have N points per unit-ish length."""
    gamma = 1.4
    nx, ny = 2 * N, N
    hx, hy = 2.0 / nx, 1.0 / ny
    g0 = Grid("outer", (nx, ny), (True, True), CARTESIAN, [BC_PERIODIC] * 4, 1, 0,
              origin=(-1.0, -0.5, 0.0), spacing=(hx, hy, hx))
    hp = 0.76 / (N - 1)
    width = 4 if sbp == 42 else 2
    margin = 6 if width == 4 else 4
    hh = 0.38 - margin * hp
    g0.holes.append(("box", (-hh, -hh), (hh, hh)))
    g1 = Grid("inner", (N, N), (False, False), CARTESIAN, [BC_INTERFACE] * 4, 1, 1,
              origin=(-0.38, -0.38, 0.0), spacing=(hp, hp, hp))
    params = default_params(gamma=gamma, Re=math.inf, sbp=sbp, order=4, hist_len=4,
                            interp_width=width, cfl=0.5)
    params["q_inf"] = [1.0, 2.0, 0.0, 1.0 / (gamma - 1.0) + 2.0, 0.0]
    q0 = []
    for g in (g0, g1):
        X = g.points()
        rho, u, v, p = vortex_state(X[0], X[1], 0.0, gamma, 5.0, 10.0, 0.0, 0.0, 2.0, 0.0)
        q0.append(conserved_from_primitive(rho, [u, v], p, gamma))
    return Workload("vortex_convergence", 2, params, [g0, g1], q0)


def periodic_curvilinear(nx: int, ny: int, amp: float = 0.08, sbp: int = 42,
                         Re: float = 50.0) -> Workload:
    """A single doubly periodic, smoothly perturbed curvilinear grid on the unit
    torus with a smooth periodic state (no holes, no boundaries)."""
    gamma = 1.4
    i = np.arange(nx)
    j = np.arange(ny)
    J, I = np.meshgrid(j, i, indexing="ij")
    xi, eta = I / nx, J / ny
    x = xi + amp * np.sin(2 * math.pi * xi) * np.sin(2 * math.pi * eta) / (2 * math.pi)
    y = eta + amp * np.sin(2 * math.pi * xi) * np.cos(2 * math.pi * eta) / (2 * math.pi)
    coords = np.stack([x.ravel(), y.ravel()])
    g = Grid("torus", (nx, ny), (True, True), CURVILINEAR, [BC_PERIODIC] * 4, 1, 0,
             coords=coords, inverse=None, coord_period=[(1.0, 0.0), (0.0, 1.0)])
    params = default_params(gamma=gamma, Re=Re, sbp=sbp, interp_width=4 if sbp == 42 else 2)
    X = coords
    rho = 1.0 + 0.2 * np.sin(2 * math.pi * X[0]) * np.cos(2 * math.pi * X[1])
    u = 0.3 + 0.1 * np.cos(2 * math.pi * X[1])
    v = -0.2 + 0.1 * np.sin(2 * math.pi * (X[0] + X[1]))
    p = 1.0 + 0.1 * np.cos(2 * math.pi * X[0])
    q0 = [conserved_from_primitive(rho, [u, v], p, gamma)]
    return Workload("periodic_curvilinear", 2, params, [g], q0)


def omesh_freestream(ntheta: int = 64, nr: int = 24, sbp: int = 42) -> Workload:
    """O-mesh alone with far-field faces at both radial ends, uniform flow."""
    gamma = 1.4
    g = omesh_grid(ntheta, nr, 1, 0, wall=False, outer_bc=BC_FARFIELD)
    params = default_params(gamma=gamma, Re=100.0, sbp=sbp, interp_width=4)
    u, v, p = 0.7, -0.3, 1.0 / gamma
    params["q_inf"] = [1.0, u, v, p / (gamma - 1.0) + 0.5 * (u * u + v * v), 0.0]
    one = np.ones(g.npts)
    q0 = [conserved_from_primitive(one, [u * one, v * one], p * one, gamma)]
    return Workload("omesh_freestream", 2, params, [g], q0)


def wall_channel(ny: int, nx: int = 8, Re: float = 100.0, mach: float = 0.2, wall_temp_ratio: float = 1.05,
                 sbp: int = 42) -> Workload:
    """Channel periodic in x with isothermal no-slip walls at y = 0 and y = 1,
    started impulsively: uniform u = 1, v = 0, rho = 1, p = 1/(gamma M^2),
    walls at wall_temp_ratio times the initial temperature."""
    gamma = 1.4
    h = 1.0 / (ny - 1)
    g = Grid("channel", (nx, ny), (True, False), CARTESIAN, [BC_PERIODIC, BC_PERIODIC, BC_WALL, BC_WALL],
             1, 0, origin=(0.0, 0.0, 0.0), spacing=(h, h, h))
    p = 1.0 / (gamma * mach * mach)
    params = default_params(gamma=gamma, Re=Re, sbp=sbp, order=4, hist_len=4,
                            interp_width=4 if sbp == 42 else 2)
    params["T_wall"] = wall_temp_ratio * p
    params["q_inf"] = [1.0, 1.0, 0.0, p / (gamma - 1.0) + 0.5, 0.0]
    one = np.ones(g.npts)
    q0 = [conserved_from_primitive(one, [one, 0.0 * one], p * one, gamma)]
    return Workload("wall_channel", 2, params, [g], q0)


def random_state_like(wl: Workload, seed: int, amp: float = 0.05) -> List[np.ndarray]:
    """Seeded smooth-free perturbation of a workload's initial state (for
    element-wise parity of one right-hand side on non-trivial data)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for q in wl.q0:
        f = 1.0 + amp * rng.uniform(-1.0, 1.0, size=q.shape)
        out.append(q * f)
    return out


CONFIGS = {
    "vortex_box": vortex_box,
    "cylinder": cylinder,
    "tgv3d": tgv3d,
}
