"""The componentwise backward-error check the GPU tests apply, pinned on the
CPU: the oracle's solutions pass it, and a solution off by one unit in the
last place in one small component (which a normwise error would not see)
fails it."""
import numpy as np

import oracle
import workloads as W
from gpuhelp import backward_error_ok


def test_oracle_solutions_pass():
    o = oracle.get()
    for T in (W.laplacian_triangle((12, 11, 10)), W.laplacian_triangle((30, 20), upper=True),
              W.powerlaw_lower(20000, 3, window=3000), W.ilu0_lower((9, 8, 7))):
        b = W.uniform_vector(T.n, 5)
        x = o.solve(T.row_ptr, T.col_idx, T.vals, b, T.upper)
        ok, worst = backward_error_ok(T, b, x)
        assert ok, (T.name, worst)


def test_small_component_error_is_caught():
    o = oracle.get()
    T = W.laplacian_triangle((12, 11, 10))
    b = W.uniform_vector(T.n, 6)
    b[17] = 1e-9                      # a tiny component
    x = o.solve(T.row_ptr, T.col_idx, T.vals, b, T.upper)
    y = x.copy()
    k = int(np.argmin(np.abs(x)))
    y[k] = x[k] * (1 + 1e-9)          # far below 1e-12 of the norm
    assert np.abs(y - x).max() / np.abs(x).max() < 1e-12
    assert not backward_error_ok(T, b, y)[0]


def test_fp32_roundoff():
    o = oracle.get()
    T = W.laplacian_triangle((10, 9, 8))
    v32 = T.vals.astype(np.float32)
    b32 = W.uniform_vector(T.n, 8).astype(np.float32)
    x = o.solve(T.row_ptr, T.col_idx, v32.astype(np.float64), b32.astype(np.float64))
    T32 = W.Triangle(T.n, T.row_ptr, T.col_idx, v32.astype(np.float64))
    assert backward_error_ok(T32, b32, x.astype(np.float32), unit_roundoff=2.0 ** -24)[0]
    # an FP32 result off by 2^-12 relative in one entry fails
    y = x.astype(np.float32)
    y[5] *= np.float32(1 + 2.0 ** -12)
    assert not backward_error_ok(T32, b32, y, unit_roundoff=2.0 ** -24)[0]
