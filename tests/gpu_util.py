"""Helpers shared by the GPU tests."""
import sys

import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_00884_amd import api
    return api


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*args):
    print("[gpu-case]", *args, file=sys.stderr, flush=True)


def close(a, b, tol, name=""):
    """Normwise relative error check with a short failure message."""
    e = rel(a, b)
    if not e < tol:
        raise AssertionError(f"{name}: normwise relative error {e:.3e} exceeds {tol:.1e}")
    return e
