"""MI355X-native multi-rate Adams-Bashforth on overset SBP-SAT meshes.

The compute path is libmrab.so (hand-written gfx950 HIP kernels behind a C
ABI, see include/mrab.h); this package is its thin Python binding plus the
host-side overset assembly.
"""
from ._lib import MrabError, load as load_library  # noqa: F401


def __getattr__(name):
    if name in ("System", "ab_coeffs"):
        from . import system
        return getattr(system, name)
    raise AttributeError(name)
