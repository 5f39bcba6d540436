"""Helpers shared by the GPU tests."""
import sys

import numpy as np


def announce(*parts):
    """Name the case on stdout before touching the GPU (flushed)."""
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def rel_max(a, b):
    """max |a - b| / max |b|"""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
