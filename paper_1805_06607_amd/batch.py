"""Many independent overset systems advanced together (C ABI mr_batch_*):
per micro-time of the batch, one work-list launch per kind of job over all
systems that step then, instead of each system's own launches."""
from __future__ import annotations

from ctypes import POINTER, byref, c_size_t, c_void_p
from typing import List

import torch

from . import _lib
from .system import System


def tile_shape_info(shape: int):
    """(tx, ty, tm) of a tile shape: tx x ty outputs per workgroup, tm
    threads per output."""
    from ctypes import c_int
    lib = _lib.load()
    tx, ty, tm = c_int(), c_int(), c_int()
    rc = lib.mr_tile_shape_info(shape, byref(tx), byref(ty), byref(tm))
    _lib.check(rc, None, "mr_tile_shape_info")
    return tx.value, ty.value, tm.value


class Batch:
    def __init__(self, systems: List[System]):
        self.lib = _lib.load()
        self.systems = list(systems)
        arr = (c_void_p * len(systems))(*[s.ctx.value for s in systems])
        self.b = c_void_p()
        rc = self.lib.mr_batch_create(arr, len(systems), byref(self.b))
        _lib.check(rc, None, "mr_batch_create")
        n = c_size_t()
        self._check(self.lib.mr_batch_workspace_size(self.b, byref(n)), "mr_batch_workspace_size")
        dev = systems[0].device
        self.ws = torch.empty(int(n.value) + 256, dtype=torch.uint8, device=dev)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self._check(self.lib.mr_batch_bind_workspace(self.b, c_void_p(base + off), c_size_t(n.value)),
                    "mr_batch_bind_workspace")

    def _check(self, rc, what):
        if rc != _lib.MR_OK:
            msg = self.lib.mr_batch_last_error(self.b).decode() if self.b else ""
            raise _lib.MrabError(f"{what}: {_lib.STATUS.get(rc, rc)} {msg}")

    def set_tile_shape(self, shape: int):
        """One tile shape for every right-hand side of the batch (-1: each
        grid's own, which keeps every system bitwise equal to its own runs)."""
        self._check(self.lib.mr_batch_set_tile_shape(self.b, shape), "mr_batch_set_tile_shape")

    def autotune(self, reps: int = 10):
        """Time every tile shape (and each grid's own) on one right-hand side
        of every grid, keep the fastest; returns (shape, {shape: ms})."""
        from ctypes import c_double, c_int
        shape = c_int()
        ms = (c_double * (_lib.NUM_TILE_SHAPES + 1))()
        self._check(self.lib.mr_batch_autotune(self.b, reps, byref(shape), ms), "mr_batch_autotune")
        return shape.value, {s - 1: ms[s] for s in range(_lib.NUM_TILE_SHAPES + 1)}

    def macrostep(self, n: int = 1):
        self._check(self.lib.mr_batch_macrostep(self.b, n), "mr_batch_macrostep")

    def close(self):
        if self.b:
            self.lib.mr_batch_destroy(self.b)
            self.b = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
