"""Helpers shared by the GPU tests: device copies of generated triangles and
error measures against the oracle."""
from __future__ import annotations

import numpy as np
import torch

DEV = "cuda:0"


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def dev_tri(T, dtype=torch.float64):
    return dev(T.row_ptr, torch.int32), dev(T.col_idx, torch.int32), dev(T.vals, dtype)


def relerr(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max()
    if den == 0:
        return float(np.abs(x).max())
    return float(np.abs(x - ref).max() / den)


def host(t):
    return t.detach().cpu().numpy()


def bits_equal(a, b):
    a = host(a) if isinstance(a, torch.Tensor) else a
    b = host(b) if isinstance(b, torch.Tensor) else b
    return np.array_equal(a.view(np.uint8), b.view(np.uint8))
