"""Shared helpers of the GPU parity tests (no method arithmetic)."""
import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # with a GPU present the HIP library must be there: import errors are failures
    from paper_1805_06607_amd import _lib
    _lib.load()
    return torch


def rel_l2(a, b, mask=None):
    """Relative L2 error per variable (rows), over the masked points."""
    a = np.asarray(a)
    b = np.asarray(b)
    if mask is not None:
        a = a[:, mask]
        b = b[:, mask]
    num = np.sqrt(np.sum((a - b) ** 2, axis=1))
    den = np.sqrt(np.sum(b ** 2, axis=1))
    return num / np.maximum(den, 1e-300)
