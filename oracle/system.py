"""One overset problem assembled for the oracle (test infrastructure only).

Builds, from a ``workloads`` problem description: blanking, runs, receivers,
donors and weights (overset.py), metric terms (exact constants on Cartesian
grids; the grid's own full-line SBP derivative of the coordinates on 2D
curvilinear grids), and exposes the coupled right-hand side used by the
integrators in integrate.py.

Donor data (section "SAT-Based Interpolation" and eq. int): at every donor
point the state q and the Cartesian viscous flux vectors F^V_j are evaluated on
the donor grid from the donor state at the receiver's time; the receiver gets
q_hat = sum_d w_d q_d and F_hat^V_j = sum_d w_d F^V_{j,d} (sum in stencil order).
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, c_double, c_int, c_int8, c_int32, c_int64
from typing import Dict, List

import numpy as np

from . import overset, sbp
from .build import LIB, build
from .integrate import MRAB

_lib = None


def load_library():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        lib = ctypes.CDLL(LIB)
        P = POINTER(OrcGridC)
        lib.orc_rhs.argtypes = [P, POINTER(c_double), POINTER(c_double), POINTER(c_double)]
        lib.orc_donor.argtypes = [P, POINTER(c_double), c_int64, POINTER(c_int64), POINTER(c_double)]
        lib.orc_dt.argtypes = [P, POINTER(c_double), POINTER(c_double)]
        lib.orc_metrics2d.argtypes = [P, POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                      POINTER(c_double), POINTER(c_double)]
        lib.orc_deriv.argtypes = [P, POINTER(c_double), c_int, POINTER(c_double)]
        lib.orc_rhs_points.argtypes = [P, POINTER(c_double), POINTER(c_double), c_int64, POINTER(c_int64),
                                       POINTER(c_double)]
        lib.orc_rhs_points.restype = c_int
        lib.orc_kmatrix.argtypes = [c_int, c_double, POINTER(c_double), POINTER(c_double), c_int,
                                    POINTER(c_double)]
        for f in (lib.orc_rhs, lib.orc_donor, lib.orc_dt, lib.orc_metrics2d, lib.orc_kmatrix,
                  lib.orc_deriv):
            f.restype = c_int
        _lib = lib
    return _lib


class OrcGridC(ctypes.Structure):
    _fields_ = [
        ("dim", c_int32), ("nv", c_int32), ("nb", c_int32), ("cw", c_int32), ("hw", c_int32),
        ("n", c_int32 * 3), ("periodic", c_int32 * 3), ("pad0", c_int32), ("npts", c_int64),
        ("dint", c_double * 5), ("dclo", (c_double * 6) * 4), ("p0", c_double),
        ("gamma", c_double), ("Re", c_double), ("Pr", c_double), ("mu", c_double), ("lam", c_double),
        ("sig_iface", c_double), ("sig_bc", c_double), ("T_wall", c_double), ("wall_visc", c_double),
        ("q_inf", c_double * 5),
        ("metric", POINTER(c_double)),
        ("pos", POINTER(c_int32) * 3), ("rlen", POINTER(c_int32) * 3),
        ("bclo", POINTER(c_int8) * 3), ("bchi", POINTER(c_int8) * 3),
        ("recv_idx", POINTER(c_int32)),
    ]


def _dp(a):
    return a.ctypes.data_as(POINTER(c_double))


def kmatrix(dim, gamma, q, nvec, sgn) -> np.ndarray:
    """K^{+} (sgn=+1) or K^{-} (sgn=-1) of the oracle, as an (nv, nv) matrix."""
    lib = load_library()
    nv = dim + 2
    q = np.ascontiguousarray(q, dtype=np.float64)
    nvec = np.ascontiguousarray(nvec, dtype=np.float64)
    out = np.zeros(nv * nv)
    rc = lib.orc_kmatrix(dim, gamma, _dp(q), _dp(nvec), int(sgn), _dp(out))
    if rc != 0:
        raise RuntimeError("orc_kmatrix failed")
    return out.reshape(nv, nv)


class _Grid:
    """Oracle-side arrays of one grid (kept alive for the C structure)."""

    def __init__(self, grid, params, iblank, run_info, metric, recv_pts):
        self.grid = grid
        self.iblank = iblank
        self.run_info = run_info
        self.metric = np.ascontiguousarray(metric)
        self.recv_pts = recv_pts
        N = grid.npts
        self.recv_idx = np.full(N, -1, dtype=np.int32)
        self.recv_idx[recv_pts] = np.arange(len(recv_pts), dtype=np.int32)
        self.struct = _make_struct(grid, params, self.metric, run_info, self.recv_idx)


def _make_struct(grid, params, metric, run_info, recv_idx) -> OrcGridC:
    s = OrcGridC()
    dim = grid.dim
    k = params["sbp"]
    interior, clo, nb, p0 = sbp.as_float_arrays(k)
    s.dim, s.nv, s.nb = dim, dim + 2, nb
    s.cw = sbp.closure_width(k)
    s.hw = sbp.table(k)["half_width"]
    n = list(grid.n) + [1] * (3 - dim)
    per = list(grid.periodic) + [False] * (3 - dim)
    for d in range(3):
        s.n[d] = n[d]
        s.periodic[d] = int(per[d])
    s.npts = grid.npts
    for i in range(5):
        s.dint[i] = interior[i]
    for i in range(4):
        for j in range(6):
            s.dclo[i][j] = clo[i][j]
    s.p0 = p0
    s.gamma, s.Re, s.Pr, s.mu = params["gamma"], params["Re"], params["Pr"], params["mu"]
    s.lam = params["lambda_over_mu"] * params["mu"]
    s.sig_iface, s.sig_bc, s.T_wall = params["sigma_I_iface"], params["sigma_I_bc"], params["T_wall"]
    s.wall_visc = params["wall_visc"]
    for i in range(5):
        s.q_inf[i] = params["q_inf"][i] if i < dim + 2 else 0.0
    s.metric = _dp(metric)
    for d in range(dim):
        pos, rlen, bclo, bchi = run_info[d]
        s.pos[d] = pos.ctypes.data_as(POINTER(c_int32))
        s.rlen[d] = rlen.ctypes.data_as(POINTER(c_int32))
        s.bclo[d] = bclo.ctypes.data_as(POINTER(c_int8))
        s.bchi[d] = bchi.ctypes.data_as(POINTER(c_int8))
    s.recv_idx = recv_idx.ctypes.data_as(POINTER(c_int32))
    return s


def cartesian_metric(grid) -> np.ndarray:
    dim = grid.dim
    N = grid.npts
    vol = 1.0
    for d in range(dim):
        vol *= grid.spacing[d]
    M = np.zeros((dim * dim + 1, N))
    for m in range(dim):
        M[m * dim + m, :] = vol / grid.spacing[m]
    M[dim * dim, :] = 1.0 / vol
    return M


def curvilinear_metric(grid, params) -> np.ndarray:
    if grid.dim != 2:
        raise NotImplementedError("curvilinear metrics are 2D only")
    lib = load_library()
    full = overset.runs(grid, np.ones(grid.npts, dtype=np.int8), params["sbp"])
    dummy = np.zeros((5, grid.npts))
    ridx = np.full(grid.npts, -1, dtype=np.int32)
    st = _make_struct(grid, params, dummy, full, ridx)
    x = np.ascontiguousarray(grid.coords[0], dtype=np.float64)
    y = np.ascontiguousarray(grid.coords[1], dtype=np.float64)
    per = grid.coord_period or [(0.0, 0.0), (0.0, 0.0)]
    perx = np.array([per[0][0], per[1][0], 0.0])
    pery = np.array([per[0][1], per[1][1], 0.0])
    out = np.zeros((5, grid.npts))
    lib.orc_metrics2d(ctypes.byref(st), _dp(x), _dp(y), _dp(perx), _dp(pery), _dp(out))
    return out


class OracleSystem:
    def __init__(self, wl):
        self.wl = wl
        self.lib = load_library()
        self.params = dict(wl.params)
        self.dim, self.nv = wl.dim, wl.dim + 2
        self.RB = self.nv + self.dim * (self.nv - 1)
        k = self.params["sbp"]
        iblanks, infos, recvs = [], [], []
        for g in wl.grids:
            ib = overset.blank(g)
            info = overset.runs(g, ib, k)
            iblanks.append(ib)
            infos.append(info)
            recvs.append(overset.receivers_fast(g, info))
        self.donor_tables = overset.donors(wl.grids, iblanks, recvs, self.params["interp_width"])
        self.grids: List[_Grid] = []
        for g, ib, info, rc in zip(wl.grids, iblanks, infos, recvs):
            M = cartesian_metric(g) if g.kind == 0 else curvilinear_metric(g, self.params)
            self.grids.append(_Grid(g, self.params, ib, info, M, rc))

    # ------------------------------------------------------------- donors
    def donor_values(self, dg: int, q: np.ndarray, pts: np.ndarray) -> np.ndarray:
        pts = np.ascontiguousarray(pts, dtype=np.int64)
        out = np.zeros((len(pts), self.RB))
        qc = np.ascontiguousarray(q, dtype=np.float64)
        rc = self.lib.orc_donor(ctypes.byref(self.grids[dg].struct), _dp(qc), len(pts),
                                pts.ctypes.data_as(POINTER(c_int64)), _dp(out))
        if rc != 0:
            raise RuntimeError("orc_donor failed")
        return out

    def _donor_arrays(self, g: int):
        """Receivers of grid g grouped by donor grid: [(dg, receiver rows,
        donor points (K, S), weights (K, S))], built once."""
        if not hasattr(self, "_darr"):
            self._darr = {}
        if g not in self._darr:
            groups: Dict[int, list] = {}
            for r, (dg, pts, wts) in enumerate(self.donor_tables[g]):
                groups.setdefault(dg, []).append((r, pts, wts))
            out = []
            for dg, items in sorted(groups.items()):
                rows = np.array([it[0] for it in items], dtype=np.int64)
                pts = np.array([it[1] for it in items], dtype=np.int64)
                wts = np.array([it[2] for it in items], dtype=np.float64)
                out.append((dg, rows, pts, wts))
            self._darr[g] = out
        return self._darr[g]

    def receiver_data(self, g: int, states: List[np.ndarray]) -> np.ndarray:
        """q_hat and F_hat^V per receiver of grid g: each receiver's weighted
        sum taken over its stencil entries in stencil order (acc = acc +
        w_e * row_e), for all receivers of one donor grid at once."""
        out = np.zeros((len(self.donor_tables[g]), self.RB))
        for dg, rows, pts, wts in self._donor_arrays(g):
            u = np.unique(pts)
            v = self.donor_values(dg, states[dg], u)
            vals = v[np.searchsorted(u, pts)]            # (K, S, RB)
            acc = np.zeros((len(rows), self.RB))
            for e in range(pts.shape[1]):
                acc = acc + wts[:, e:e + 1] * vals[:, e, :]
            out[rows] = acc
        return out

    def receiver_data_loop(self, g: int, states: List[np.ndarray]) -> np.ndarray:
        """receiver_data written receiver by receiver (the plain loop)."""
        entries = self.donor_tables[g]
        out = np.zeros((len(entries), self.RB))
        if not entries:
            return out
        by_donor: Dict[int, list] = {}
        for e in entries:
            by_donor.setdefault(e[0], []).extend(e[1])
        vals = {}
        for dg, pts in by_donor.items():
            u = np.unique(np.array(pts, dtype=np.int64))
            v = self.donor_values(dg, states[dg], u)
            vals[dg] = (u, v)
        for r, (dg, pts, wts) in enumerate(entries):
            u, v = vals[dg]
            rows = v[np.searchsorted(u, pts)]
            acc = np.zeros(self.RB)
            for e in range(len(pts)):
                acc = acc + wts[e] * rows[e]
            out[r] = acc
        return out

    # ---------------------------------------------------------------- rhs
    def rhs_grid(self, g: int, q: np.ndarray, recv: np.ndarray) -> np.ndarray:
        qc = np.ascontiguousarray(q, dtype=np.float64).reshape(self.nv, -1)
        rb = np.ascontiguousarray(recv, dtype=np.float64)
        if rb.size == 0:
            rb = np.zeros((1, self.RB))
        out = np.zeros_like(qc)
        rc = self.lib.orc_rhs(ctypes.byref(self.grids[g].struct), _dp(qc), _dp(rb), _dp(out))
        if rc != 0:
            raise RuntimeError(f"orc_rhs failed ({rc})")
        return out

    def rhs_points(self, g: int, q: np.ndarray, recv: np.ndarray, pts) -> np.ndarray:
        """Right-hand side of grid g at the listed points only, (len(pts), nv)."""
        qc = np.ascontiguousarray(q, dtype=np.float64).reshape(self.nv, -1)
        rb = np.ascontiguousarray(recv, dtype=np.float64)
        if rb.size == 0:
            rb = np.zeros((1, self.RB))
        pts = np.ascontiguousarray(pts, dtype=np.int64)
        out = np.zeros((len(pts), self.nv))
        rc = self.lib.orc_rhs_points(ctypes.byref(self.grids[g].struct), _dp(qc), _dp(rb), len(pts),
                                     pts.ctypes.data_as(POINTER(c_int64)), _dp(out))
        if rc != 0:
            raise RuntimeError(f"orc_rhs_points failed ({rc})")
        return out

    def rhs(self, states: List[np.ndarray], which=None) -> Dict[int, np.ndarray]:
        which = range(len(self.grids)) if which is None else which
        out = {}
        for g in which:
            out[g] = self.rhs_grid(g, states[g], self.receiver_data(g, states))
        return out

    def deriv(self, g: int, f: np.ndarray, d: int) -> np.ndarray:
        """D along direction d of a scalar field on grid g (runs with closures)."""
        fc = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(self.grids[g].grid.npts)
        self.lib.orc_deriv(ctypes.byref(self.grids[g].struct), _dp(fc), d, _dp(out))
        return out

    # ---------------------------------------------------------- timestep
    def dt_points(self, g: int, q: np.ndarray) -> np.ndarray:
        qc = np.ascontiguousarray(q, dtype=np.float64)
        out = np.zeros(self.grids[g].grid.npts)
        self.lib.orc_dt(ctypes.byref(self.grids[g].struct), _dp(qc), _dp(out))
        return out

    def timestep(self, states=None):
        """(h, H): H = cfl * min over levels of rate * min_pt dt (or dt_fixed);
        h = H / r_max."""
        states = states if states is not None else self.wl.q0
        rates = [g.rate for g in self.wl.grids]
        rmax = max(rates)
        if self.params.get("dt_fixed", 0.0) > 0.0:
            H = float(self.params["dt_fixed"])
        else:
            H = math.inf
            for g, q in enumerate(states):
                H = min(H, rates[g] * float(np.min(self.dt_points(g, q))))
            H = self.params["cfl"] * H
        return H / rmax, H

    def integrator(self, H=None) -> MRAB:
        if H is None:
            H = self.timestep()[1]
        rates = [g.rate for g in self.wl.grids]
        return MRAB(self.rhs, rates, self.params["order"], self.params["hist_len"], H)

    @property
    def active_masks(self):
        return [gr.iblank.astype(bool) for gr in self.grids]
