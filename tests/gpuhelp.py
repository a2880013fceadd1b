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


def backward_error_ok(T, b, x, unit_roundoff=2.0 ** -53, extra=2):
    """Componentwise backward stability of a computed solution (Higham,
    Accuracy and Stability of Numerical Algorithms, Thm 8.5): with the
    residual r = b - T x^ and s = |T||x^| computed in extended precision,
    |r_i| <= gamma_{m_i + extra} s_i for m_i the stored entries of row i.
    extra = 2 covers the kernels' reciprocal of the diagonal (one rounding
    for 1/d, one for the product) on top of the substitution's m_i roundings;
    any summation order and FMA stay inside the bound.  Scale-free: small
    components are held to their own residual, unlike a normwise error.
    Returns (ok, worst ratio |r_i| / (gamma s_i))."""
    rows = np.repeat(np.arange(T.n), np.diff(T.row_ptr))
    v = np.asarray(T.vals).astype(np.longdouble)
    xl = np.asarray(x).astype(np.longdouble)
    prod = v * xl[T.col_idx]
    r = np.asarray(b).astype(np.longdouble).copy()
    np.subtract.at(r, rows, prod)
    s = np.zeros(T.n, dtype=np.longdouble)
    np.add.at(s, rows, np.abs(prod))
    m = np.diff(T.row_ptr).astype(np.float64) + extra
    gam = m * unit_roundoff / (1 - m * unit_roundoff)
    lim = gam * s
    ratio = np.where(lim > 0, np.abs(r) / np.where(lim > 0, lim, 1), np.where(r == 0, 0, np.inf))
    worst = float(ratio.max()) if T.n else 0.0
    return worst <= 1.0, worst
