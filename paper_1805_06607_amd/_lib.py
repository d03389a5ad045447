"""ctypes binding of libmrab.so (argument marshalling only).

The library is built in-tree by ``paper_1805_06607_amd.build``; importing the
binding without it raises immediately: there is no fallback path.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int8, c_int64, c_size_t, c_void_p, c_char_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrab.so")

MR_OK = 0
NUM_TILE_SHAPES = 8          # MR_NUM_TILE_SHAPES of mrab.h
STATUS = {0: "MR_OK", -1: "MR_ERR_ARG", -2: "MR_ERR_STATE", -3: "MR_ERR_SETUP", -4: "MR_ERR_HIP",
          -5: "MR_ERR_NONFINITE", -6: "MR_ERR_UNSUPPORTED"}


class MrParams(ctypes.Structure):
    _fields_ = [
        ("dim", c_int), ("sbp", c_int), ("order", c_int), ("hist_len", c_int), ("interp_width", c_int),
        ("gamma", c_double), ("Re", c_double), ("Pr", c_double), ("mu", c_double), ("lambda_over_mu", c_double),
        ("sigma_I_iface", c_double), ("sigma_I_bc", c_double), ("T_wall", c_double), ("wall_visc", c_double),
        ("q_inf", c_double * 5), ("cfl", c_double), ("dt_fixed", c_double),
    ]


class MrGridDesc(ctypes.Structure):
    _fields_ = [
        ("n", c_int * 3), ("periodic", c_int * 3), ("kind", c_int),
        ("origin", c_double * 3), ("spacing", c_double * 3),
        ("coords", POINTER(c_double)), ("coord_period", (c_double * 3) * 3),
        ("iblank", POINTER(c_int8)), ("face_bc", c_int * 6), ("rate", c_int),
    ]


# mr_locate_fn of mrab.h
LOCATE_FN = ctypes.CFUNCTYPE(c_int, c_void_p, c_int, c_int64, POINTER(c_double), POINTER(c_double))


class MrabError(RuntimeError):
    pass


_lib = None

SIGNATURES = {
    "mr_create": [POINTER(MrParams), c_void_p, POINTER(c_void_p)],
    "mr_add_grid": [c_void_p, POINTER(MrGridDesc), POINTER(c_int)],
    "mr_set_overset": [c_void_p, c_int, c_int, c_int64, c_int, POINTER(c_int64), POINTER(c_int64),
                       POINTER(c_double)],
    "mr_assemble_overset": [c_void_p, c_int, POINTER(c_int), LOCATE_FN, c_void_p],
    "mr_get_overset": [c_void_p, c_int, POINTER(c_int64), POINTER(c_int64), POINTER(c_int), POINTER(c_int64),
                       POINTER(c_double)],
    "mr_finalize": [c_void_p, POINTER(c_size_t)],
    "mr_bind_workspace": [c_void_p, c_void_p, c_size_t],
    "mr_bind_static_workspace": [c_void_p],
    "mr_set_state": [c_void_p, c_int, c_void_p],
    "mr_get_state": [c_void_p, c_int, c_void_p],
    "mr_rhs": [c_void_p, c_double, POINTER(c_void_p), POINTER(c_void_p)],
    "mr_receiver_data": [c_void_p, c_int, POINTER(c_void_p), c_void_p],
    "mr_num_receivers": [c_void_p, c_int, POINTER(c_int64)],
    "mr_timestep": [c_void_p, POINTER(c_double), POINTER(c_double)],
    "mr_mrab_start": [c_void_p, c_double],
    "mr_mrab_macrostep": [c_void_p, c_int],
    "mr_get_history": [c_void_p, c_int, c_int, c_void_p],
    "mr_set_history": [c_void_p, c_int, c_int, c_void_p],
    "mr_set_macrostep": [c_void_p, c_double],
    "mr_mrab_resume": [c_void_p, c_double],
    "mr_time": [c_void_p, POINTER(c_double), POINTER(c_int64)],
    "mr_ab_coeffs": [c_int, c_int, c_double, c_double, POINTER(c_double)],
    "mr_kernel_timing": [c_void_p, c_int, c_int],
    "mr_kernel_time": [c_void_p, POINTER(c_double), POINTER(c_int)],
    "mr_kernel_time_grid": [c_void_p, c_int, POINTER(c_double), POINTER(c_int)],
    "mr_set_option": [c_void_p, c_char_p, c_int64],
    "mr_set_tile_shape": [c_void_p, c_int, c_int],
    "mr_get_tile_shape": [c_void_p, c_int, POINTER(c_int), POINTER(c_int), POINTER(c_int), POINTER(c_int)],
    "mr_tile_shape_info": [c_int, POINTER(c_int), POINTER(c_int), POINTER(c_int)],
    "mr_autotune": [c_void_p, c_int],
    "mr_guard": [c_void_p, POINTER(c_double)],
    "mr_batch_create": [POINTER(c_void_p), c_int, POINTER(c_void_p)],
    "mr_batch_workspace_size": [c_void_p, POINTER(c_size_t)],
    "mr_batch_bind_workspace": [c_void_p, c_void_p, c_size_t],
    "mr_batch_macrostep": [c_void_p, c_int],
    "mr_batch_set_tile_shape": [c_void_p, c_int],
    "mr_batch_autotune": [c_void_p, c_int, POINTER(c_int), POINTER(c_double)],
    "mr_batch_last_error": [c_void_p],
    "mr_batch_destroy": [c_void_p],
    "mr_save_bytes": [c_void_p, POINTER(c_size_t)],
    "mr_save": [c_void_p, c_void_p, c_size_t],
    "mr_load": [c_void_p, c_void_p, c_size_t],
    "mr_adj_set_objective": [c_void_p, c_int, c_int64, POINTER(c_int64), POINTER(c_double)],
    "mr_adj_workspace_size": [c_void_p, c_int, POINTER(c_size_t)],
    "mr_adj_bind_workspace": [c_void_p, c_void_p, c_size_t],
    "mr_adj_rhs": [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p)],
    "mr_adj_forward": [c_void_p, c_int, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_double)],
    "mr_adj_gradient": [c_void_p, c_int, POINTER(c_void_p), POINTER(c_void_p), c_double, POINTER(c_void_p),
                        POINTER(c_double), POINTER(c_int64)],
    "mr_adj_schedule": [c_int, c_int, POINTER(c_int64)],
    "mr_last_error": [c_void_p],
    "mr_destroy": [c_void_p],
}


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1805_06607_amd.build` "
                "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        lib = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = c_int
        lib.mr_last_error.restype = c_char_p
        lib.mr_destroy.restype = None
        lib.mr_batch_last_error.restype = c_char_p
        lib.mr_batch_destroy.restype = None
        _lib = lib
    return _lib


def check(rc, ctx=None, what=""):
    if rc != MR_OK:
        msg = ""
        if ctx is not None:
            msg = load().mr_last_error(ctx).decode()
        raise MrabError(f"{what}: {STATUS.get(rc, rc)} {msg}")
