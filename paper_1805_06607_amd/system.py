"""Python front end of libmrab.so: one overset system on one GPU.

PyTorch provides the device memory (one workspace tensor, the state tensors)
and the stream; every step of the right-hand side and of the time integration
runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, byref, c_double, c_int, c_int8, c_int64, c_size_t, c_void_p
from typing import List, Optional

import numpy as np
import torch

from . import _lib
from . import assemble

CART, CURV = 0, 1


def _params(wl) -> _lib.MrParams:
    P = wl.params
    p = _lib.MrParams()
    p.dim = wl.dim
    p.sbp = int(P["sbp"])
    p.order = int(P["order"])
    p.hist_len = int(P["hist_len"])
    p.interp_width = int(P["interp_width"])
    p.gamma, p.Re, p.Pr, p.mu = P["gamma"], P["Re"], P["Pr"], P["mu"]
    p.lambda_over_mu = P["lambda_over_mu"]
    p.sigma_I_iface, p.sigma_I_bc = P["sigma_I_iface"], P["sigma_I_bc"]
    p.T_wall, p.wall_visc = P["T_wall"], P["wall_visc"]
    for i in range(5):
        p.q_inf[i] = P["q_inf"][i] if i < len(P["q_inf"]) else 0.0
    p.cfl = P["cfl"]
    p.dt_fixed = P.get("dt_fixed", 0.0)
    return p


class HostSetup:
    """A problem's host-side setup through the C ABI (no device touched):
    context, grids (blanking from the problem's hole shapes), the library's
    donor search and weights; the receiver rows and donor stencils read back.
    ``stream`` is a hipStream_t handle (None: the default stream).  With
    ``own_locate`` the library locates points in curvilinear grids by its own
    search instead of the problem's closed-form inverse map."""

    def __init__(self, wl, stream=None, own_locate: bool = False):
        self.own_locate = own_locate
        self.lib = _lib.load()
        self.wl = wl
        self.dim = wl.dim
        self._params = _params(wl)
        self.ctx = c_void_p()
        _lib.check(self.lib.mr_create(byref(self._params), c_void_p(stream), byref(self.ctx)), None, "mr_create")
        try:
            self._grids_and_overset(wl)
        except Exception:
            self.lib.mr_destroy(self.ctx)
            self.ctx = c_void_p()
            raise

    def _check(self, rc, what):
        _lib.check(rc, self.ctx, what)

    def _grids_and_overset(self, wl):
        self.iblanks = []
        self._keep = []
        for g in wl.grids:
            ib = assemble.iblank(g)
            self.iblanks.append(ib)
            d = _lib.MrGridDesc()
            for k in range(3):
                d.n[k] = g.n[k] if k < g.dim else 1
                d.periodic[k] = int(g.periodic[k]) if k < g.dim else 0
                d.origin[k] = g.origin[k] if k < len(g.origin) else 0.0
                d.spacing[k] = g.spacing[k] if k < len(g.spacing) else 1.0
            d.kind = CURV if g.kind == 1 else CART
            if g.kind == 1:
                coords = np.ascontiguousarray(g.coords, dtype=np.float64)
                self._keep.append(coords)
                d.coords = coords.ctypes.data_as(POINTER(c_double))
                per = g.coord_period or [(0.0, 0.0), (0.0, 0.0)]
                for a in range(len(per)):
                    for b in range(len(per[a])):
                        d.coord_period[a][b] = per[a][b]
            self._keep.append(ib)
            d.iblank = ib.ctypes.data_as(POINTER(c_int8))
            for k in range(2 * g.dim):
                d.face_bc[k] = g.face_bc[k]
            d.rate = g.rate
            gid = c_int()
            self._check(self.lib.mr_add_grid(self.ctx, byref(d), byref(gid)), "mr_add_grid")

        # donor search and weights in the library; curvilinear grids located
        # by the problem description's closed-form inverse map (or the
        # library's own search)
        W = int(wl.params["interp_width"])
        dim = self.dim

        def locate(_user, grid, n, x, f):
            try:
                if n > 0:
                    X = np.ctypeslib.as_array(x, shape=(dim * n,)).reshape(dim, n)
                    out = np.ctypeslib.as_array(f, shape=(dim * n,))
                    out[:] = np.asarray(wl.grids[grid].frac_index(X), dtype=np.float64).reshape(-1)
                return 0
            except Exception:
                return 1

        self._locate = _lib.LOCATE_FN() if self.own_locate else _lib.LOCATE_FN(locate)
        prio = (c_int * len(wl.grids))(*[int(g.priority) for g in wl.grids])
        self._check(self.lib.mr_assemble_overset(self.ctx, W, prio, self._locate, None), "mr_assemble_overset")
        S = W ** self.dim
        # the library's receiver rows (registration order) and donor stencils
        self.recv_pts, self.donor_tables, self.recv_order = [], [], []
        for g in range(len(wl.grids)):
            n = c_int64()
            self._check(self.lib.mr_get_overset(self.ctx, g, byref(n), None, None, None, None), "mr_get_overset")
            k = int(n.value)
            rp = np.zeros(max(k, 1), dtype=np.int64)
            dg = np.zeros(max(k, 1), dtype=np.int32)
            pts = np.zeros(max(k, 1) * S, dtype=np.int64)
            w = np.zeros(max(k, 1) * S, dtype=np.float64)
            self._check(self.lib.mr_get_overset(self.ctx, g, byref(n), rp.ctypes.data_as(POINTER(c_int64)),
                                                dg.ctypes.data_as(POINTER(c_int)),
                                                pts.ctypes.data_as(POINTER(c_int64)),
                                                w.ctypes.data_as(POINTER(c_double))), "mr_get_overset")
            rp, dg, pts, w = rp[:k], dg[:k], pts[:k * S].reshape(k, S), w[:k * S].reshape(k, S)
            self.recv_order.append(rp.copy())
            self.recv_pts.append(np.sort(rp))
            tab = {}
            for d in dict.fromkeys(dg.tolist()):
                sel = dg == d
                tab[int(d)] = (rp[sel], pts[sel], w[sel])
            self.donor_tables.append(tab)


class System:
    """An overset problem assembled on the GPU.

    ``wl`` is a problem description (see the ``workloads`` package): grids,
    boundary flags, hole shapes, rates, parameters and initial states.
    """

    def __init__(self, wl, device: str = "cuda:0", stream: Optional[torch.cuda.Stream] = None,
                 static_workspace: bool = False):
        self.lib = _lib.load()
        self.wl = wl
        self.device = torch.device(device)
        self.dim, self.nv = wl.dim, wl.dim + 2
        self.RB = self.nv + self.dim * (self.nv - 1)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._host = HostSetup(wl, self.stream.cuda_stream)
        self.ctx = self._host.ctx
        self._params = self._host._params
        self.iblanks = self._host.iblanks
        self.recv_pts = self._host.recv_pts
        self.donor_tables = self._host.donor_tables
        self.recv_order = self._host.recv_order
        nbytes = c_size_t()
        self._check(self.lib.mr_finalize(self.ctx, byref(nbytes)), "mr_finalize")
        self.workspace_bytes = int(nbytes.value)
        if static_workspace:
            # the library's own per-device array: no device allocation here
            self.ws = None
            with torch.cuda.device(self.device):
                self._check(self.lib.mr_bind_static_workspace(self.ctx), "mr_bind_static_workspace")
        else:
            self.ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=self.device)
            base = self.ws.data_ptr()
            off = (-base) % 256
            self._check(self.lib.mr_bind_workspace(self.ctx, c_void_p(base + off), c_size_t(nbytes.value)),
                        "mr_bind_workspace")
        self.set_states([torch.as_tensor(q, dtype=torch.float64) for q in wl.q0])

    # ------------------------------------------------------------ helpers
    def _check(self, rc, what):
        _lib.check(rc, self.ctx, what)

    def _dev(self, q) -> torch.Tensor:
        t = torch.as_tensor(q, dtype=torch.float64)
        return t.to(self.device).contiguous()

    @property
    def ngrids(self):
        return len(self.wl.grids)

    def npts(self, g):
        return self.wl.grids[g].npts

    # -------------------------------------------------------------- state
    def set_states(self, states: List) -> None:
        self._states_keep = [self._dev(q).reshape(self.nv, -1) for q in states]
        for g, t in enumerate(self._states_keep):
            self._check(self.lib.mr_set_state(self.ctx, g, c_void_p(t.data_ptr())), "mr_set_state")

    def state(self, g: int) -> torch.Tensor:
        out = torch.empty((self.nv, self.npts(g)), dtype=torch.float64, device=self.device)
        self._check(self.lib.mr_get_state(self.ctx, g, c_void_p(out.data_ptr())), "mr_get_state")
        return out

    # ---------------------------------------------------------------- rhs
    def rhs(self, states: List, t: float = 0.0) -> List[torch.Tensor]:
        qs = [self._dev(q).reshape(self.nv, -1) for q in states]
        outs = [torch.empty_like(q) for q in qs]
        qa = (c_void_p * len(qs))(*[q.data_ptr() for q in qs])
        oa = (c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        self._check(self.lib.mr_rhs(self.ctx, t, qa, oa), "mr_rhs")
        self._alive = (qs, outs)
        return outs

    def receiver_data(self, g: int, states: List) -> torch.Tensor:
        """Receiver rows of grid g, in ascending receiver point order."""
        qs = [self._dev(q).reshape(self.nv, -1) for q in states]
        n = c_int64()
        self._check(self.lib.mr_num_receivers(self.ctx, g, byref(n)), "mr_num_receivers")
        out = torch.zeros((max(n.value, 1), self.RB), dtype=torch.float64, device=self.device)
        qa = (c_void_p * len(qs))(*[q.data_ptr() for q in qs])
        self._check(self.lib.mr_receiver_data(self.ctx, g, qa, c_void_p(out.data_ptr())), "mr_receiver_data")
        self._alive = (qs, out)
        out = out[: n.value]
        perm = np.argsort(self.recv_order[g], kind="stable")
        return out[torch.as_tensor(perm, device=self.device)]

    # --------------------------------------------------------- integrate
    def timestep(self):
        h, H = c_double(), c_double()
        self._check(self.lib.mr_timestep(self.ctx, byref(h), byref(H)), "mr_timestep")
        return h.value, H.value

    def set_macrostep(self, H: float):
        """Fix the macrostep H (h = H / r_max) instead of the estimate."""
        self._check(self.lib.mr_set_macrostep(self.ctx, H), "mr_set_macrostep")

    def start(self, t0: float = 0.0):
        self._check(self.lib.mr_mrab_start(self.ctx, t0), "mr_mrab_start")

    def macrostep(self, n: int = 1):
        self._check(self.lib.mr_mrab_macrostep(self.ctx, n), "mr_mrab_macrostep")

    def set_history(self, g: int, j: int, F) -> None:
        """History value j (0 oldest .. m-1 newest) of grid g."""
        t = self._dev(F).reshape(self.nv, -1)
        self._hist_keep = getattr(self, "_hist_keep", {})
        self._hist_keep[(g, j)] = t
        self._check(self.lib.mr_set_history(self.ctx, g, j, c_void_p(t.data_ptr())), "mr_set_history")

    def resume(self, t: float = 0.0):
        """Continue MRAB from the current states and histories at time t."""
        self._check(self.lib.mr_mrab_resume(self.ctx, t), "mr_mrab_resume")

    def history(self, g: int, j: int) -> torch.Tensor:
        out = torch.empty((self.nv, self.npts(g)), dtype=torch.float64, device=self.device)
        self._check(self.lib.mr_get_history(self.ctx, g, j, c_void_p(out.data_ptr())), "mr_get_history")
        return out

    def time(self):
        t, k = c_double(), c_int64()
        self._check(self.lib.mr_time(self.ctx, byref(t), byref(k)), "mr_time")
        return t.value, k.value

    def guard(self) -> float:
        v = c_double()
        self._check(self.lib.mr_guard(self.ctx, byref(v)), "mr_guard")
        return v.value

    def kernel_timing(self, grid: int, max_events: int):
        """Time the fused right-hand-side launches of one grid (-2: all grids)."""
        self._check(self.lib.mr_kernel_timing(self.ctx, grid, max_events), "mr_kernel_timing")

    def kernel_time(self, grid: int = -1):
        """(summed ms, launches) of the timed launches (grid -1: all grids)."""
        ms, n = c_double(), c_int()
        self._check(self.lib.mr_kernel_time_grid(self.ctx, grid, byref(ms), byref(n)), "mr_kernel_time_grid")
        return ms.value, n.value

    def set_option(self, name: str, value: int):
        """Launch-plan option ("rhs_two_pass")."""
        self._check(self.lib.mr_set_option(self.ctx, name.encode(), int(value)), "mr_set_option")

    def save(self) -> torch.Tensor:
        """Checkpoint of the integrator (states, histories, time, macrosteps,
        H) in a new device tensor."""
        n = c_size_t()
        self._check(self.lib.mr_save_bytes(self.ctx, byref(n)), "mr_save_bytes")
        buf = torch.empty(int(n.value), dtype=torch.uint8, device=self.device)
        self._check(self.lib.mr_save(self.ctx, c_void_p(buf.data_ptr()), c_size_t(n.value)), "mr_save")
        return buf

    def load(self, buf: torch.Tensor) -> None:
        """Restart from a checkpoint made by save() (this or another System
        of the same problem)."""
        b = buf.to(self.device).contiguous()
        self._check(self.lib.mr_load(self.ctx, c_void_p(b.data_ptr()), c_size_t(b.numel())), "mr_load")

    def set_tile_shape(self, grid: int, shape: int):
        """Tile shape of a 2D grid's fused kernel (-1: size-based default)."""
        self._check(self.lib.mr_set_tile_shape(self.ctx, grid, shape), "mr_set_tile_shape")

    def tile_shape(self, grid: int):
        """(shape, tx, ty, tm) in use for a grid; shape -1 for 3D grids."""
        s, tx, ty, tm = c_int(), c_int(), c_int(), c_int()
        self._check(self.lib.mr_get_tile_shape(self.ctx, grid, byref(s), byref(tx), byref(ty), byref(tm)),
                    "mr_get_tile_shape")
        return s.value, tx.value, ty.value, tm.value

    def autotune(self, reps: int = 20):
        """Time every tile shape on each 2D grid and keep the fastest."""
        self._check(self.lib.mr_autotune(self.ctx, reps), "mr_autotune")
        return [self.tile_shape(g) for g in range(self.ngrids)]

    def close(self):
        if self.ctx:
            self.lib.mr_destroy(self.ctx)
            self.ctx = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ab_coeffs(order: int, hist_len: int, tau: float = 1.0, spacing: float = 1.0) -> np.ndarray:
    """spacing * alpha_j (oldest first) of mr_ab_coeffs."""
    out = (c_double * hist_len)()
    _lib.check(_lib.load().mr_ab_coeffs(order, hist_len, spacing, tau, out), None, "mr_ab_coeffs")
    return np.array(out[:])
