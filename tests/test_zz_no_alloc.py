"""sptrsv_solve_noalloc (the allocation-free solve) through the C ABI.

Its output must equal sptrsv_solve's bit for bit (same schedule, same
kernels; only the position-ordered scratch differs) and match the oracle
within the FP64 tolerance, on two calls in a row, the second with a smaller
triangle, and again on the first after the array held the second's values.
Sizes beyond the fixed scratch capacity, and schedules whose work tables
were never built, are refused with their own status codes.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpuhelp import DEV, bits_equal, dev, dev_tri, host, relerr

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module")
def sp():
    import paper_1710_04985_amd as sp
    assert torch.cuda.is_available()
    return sp


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _noalloc(sp, h, b, x):
    return sp.lib.sptrsv_solve_noalloc(h._h, ctypes.c_void_p(b.data_ptr()),
                                       ctypes.c_void_p(x.data_ptr()), _stream())


def _case(sp, T, seed, **opts):
    h = sp.Handle(*dev_tri(T), uplo="U" if T.upper else "L")
    if opts:
        h.configure(**opts)
    b = W.uniform_vector(T.n, seed)
    bd = dev(b)
    xo = oracle.get().solve(T.row_ptr, T.col_idx, T.vals, b, T.upper)
    return h, bd, xo


def test_noalloc_matches_solve_two_calls(sp):
    big = W.laplacian_triangle((48, 48, 48))                 # 110,592 rows, 142 levels
    small = W.c1_lap2d_64()[0]                               # 4,096 rows, 127 levels
    h1, b1, xo1 = _case(sp, big, 11)
    h2, b2, xo2 = _case(sp, small, 12)
    ref1 = h1.solve(b1)
    ref2 = h2.solve(b2)
    x1 = torch.full_like(b1, float("nan"))
    x2 = torch.full_like(b2, float("nan"))
    print("noalloc: 48^3 lower, then 64x64 lower, then 48^3 again", flush=True)
    assert _noalloc(sp, h1, b1, x1) == 0
    h1.status()
    assert bits_equal(x1, ref1)
    assert relerr(host(x1), xo1) <= TOL64
    assert _noalloc(sp, h2, b2, x2) == 0                     # smaller input, same array
    h2.status()
    assert bits_equal(x2, ref2)
    assert relerr(host(x2), xo2) <= TOL64
    x1.fill_(float("nan"))
    assert _noalloc(sp, h1, b1, x1) == 0                     # array holds the small solve's values
    h1.status()
    assert bits_equal(x1, ref1)


@pytest.mark.parametrize("opts", [dict(algo=1), dict(algo=2, assign=1), dict(algo=2, sync=1),
                                  dict(algo=2, assign=2, grid=16), dict(algo=2, xp_stride=4)])
def test_noalloc_other_schedules(sp, opts):
    T = W.laplacian_triangle((20, 20, 20), upper=True)
    h, bd, xo = _case(sp, T, 13, **opts)
    ref = h.solve(bd)                                        # builds this schedule's tables
    x = torch.full_like(bd, float("nan"))
    assert _noalloc(sp, h, bd, x) == 0
    h.status()
    assert bits_equal(x, ref)
    assert relerr(host(x), xo) <= TOL64


def test_noalloc_in_place(sp):
    T = W.laplacian_triangle((24, 16, 12))
    h, bd, xo = _case(sp, T, 14)
    x = bd.clone()
    assert _noalloc(sp, h, x, x) == 0
    h.status()
    assert relerr(host(x), xo) <= TOL64


def test_noalloc_refuses_oversize_and_unprepared(sp):
    # 84^3 = 592,704 rows in 128-byte slots need 75.9 MB > 64 MiB
    T = W.laplacian_triangle((84, 84, 84))
    h, bd, xo = _case(sp, T, 15)
    h.set_option("xp_stride", 16)             # a slot width asks for a static schedule
    x = torch.empty_like(bd)
    h.solve(bd, out=x)                        # builds that schedule's per-wavefront lists
    assert _noalloc(sp, h, bd, x) == -13                     # SPTRSV_ERR_TOO_LARGE
    h.set_option("xp_stride", 1)
    assert _noalloc(sp, h, bd, x) == 0
    h.status()
    assert relerr(host(x), xo) <= TOL64
    # a column-wise schedule whose push lists were never built: refused, not built
    T2 = W.laplacian_triangle((10, 10, 10))
    h2, b2, _ = _case(sp, T2, 16, algo=5)
    assert _noalloc(sp, h2, b2, torch.empty_like(b2)) == -11   # SPTRSV_ERR_NOT_SUPPORTED
    # the transposed analysis is not built by it either: a later plain solve still works
    h2.configure(algo=2)
    x2 = torch.empty_like(b2)
    assert _noalloc(sp, h2, b2, x2) == 0
    h2.status()
