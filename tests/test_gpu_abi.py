"""The boundary's literal entry points, called through ctypes exactly as the
C header declares them: sptrsv_analyze (the problem statement's analysis
call, host route), sptrsv_export_analysis, sptrsv_get_info, sptrsv_solve,
sptrsv_solve_transpose, sptrsv_solve_multi, sptrsv_get_status and
sptrsv_destroy.  Analysis bit-exact against the oracle, solves within the
FP64 tolerance, validation errors reported with their codes."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpuhelp import dev, dev_tri, host, relerr

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
P32 = ctypes.POINTER(ctypes.c_int32)


@pytest.fixture(scope="module")
def lib():
    import paper_1710_04985_amd as sp
    assert torch.cuda.is_available()
    return sp.lib


def _s():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _ip(a):
    return a.ctypes.data_as(P32)


@pytest.mark.parametrize("T", [W.laplacian_triangle((20, 19, 18)),
                               W.laplacian_triangle((20, 19, 18), upper=True),
                               W.powerlaw_lower(30000, 4, window=3000), W.ilu0_lower((8, 8, 8))],
                         ids=lambda t: t.name)
def test_sptrsv_analyze_literal(lib, T):
    o = oracle.get()
    rp, ci, v = dev_tri(T)
    h = ctypes.c_void_p()
    assert lib.sptrsv_analyze(T.n, T.nnz, _p(rp), _p(ci), _p(v), 0, int(T.upper), 0, _s(),
                              ctypes.byref(h)) == 0
    level = np.zeros(T.n, np.int32)
    ilev = np.zeros(T.n + 1, np.int32)
    jlev = np.zeros(T.n, np.int32)
    dep = np.zeros(T.n, np.int32)
    assert lib.sptrsv_export_analysis(h, 0, _ip(level), _ip(ilev), _ip(jlev), _ip(dep)) == 0
    lv, nlev, ilev_o, jlev_o, dep_o = o.analyze(T.row_ptr, T.col_idx, T.upper)
    assert np.array_equal(level, lv)
    assert np.array_equal(ilev[:nlev + 1], ilev_o)
    assert np.array_equal(jlev, jlev_o)
    assert np.array_equal(dep, dep_o)
    n_out, nlev_out, algo, group = (ctypes.c_int32() for _ in range(4))
    nnz_out = ctypes.c_int64()
    assert lib.sptrsv_get_info(h, ctypes.byref(n_out), ctypes.byref(nnz_out),
                               ctypes.byref(nlev_out), ctypes.byref(algo),
                               ctypes.byref(group)) == 0
    assert (n_out.value, nnz_out.value, nlev_out.value) == (T.n, T.nnz, nlev)
    b = W.uniform_vector(T.n, 41)
    bd = dev(b)
    x = torch.empty_like(bd)
    assert lib.sptrsv_solve(h, _p(bd), _p(x), _s()) == 0
    assert lib.sptrsv_get_status(h) == 0
    assert relerr(host(x), o.solve(T.row_ptr, T.col_idx, T.vals, b, T.upper)) <= TOL64
    assert lib.sptrsv_solve_transpose(h, _p(bd), _p(x), _s()) == 0
    assert lib.sptrsv_get_status(h) == 0
    assert relerr(host(x), o.solve_transpose(T.row_ptr, T.col_idx, T.vals, b, T.upper)) <= TOL64
    F = np.stack([W.uniform_vector(T.n, 50 + r) for r in range(3)], 0)
    Fd = dev(F)
    X = torch.empty_like(Fd)
    assert lib.sptrsv_solve_multi(h, 3, T.n, _p(Fd), _p(X), 0, _s()) == 0
    assert lib.sptrsv_get_status(h) == 0
    Xo = o.solve_multi(T.row_ptr, T.col_idx, T.vals, F.T, T.upper)
    assert relerr(host(X).T, Xo) <= TOL64
    assert lib.sptrsv_destroy(h) == 0


def test_sptrsv_analyze_literal_errors(lib):
    T = W.laplacian_triangle((5, 4, 3))
    rp, ci, v = dev_tri(T)
    h = ctypes.c_void_p()
    # the lower pattern analysed as upper: entries on the wrong side
    assert lib.sptrsv_analyze(T.n, T.nnz, _p(rp), _p(ci), _p(v), 0, 1, 0, _s(),
                              ctypes.byref(h)) == -4
    assert not h.value
    # a zero pivot
    v0 = v.clone()
    v0[T.row_ptr[3] + int(np.flatnonzero(T.col_idx[T.row_ptr[3]:T.row_ptr[4]] == 3)[0])] = 0.0
    assert lib.sptrsv_analyze(T.n, T.nnz, _p(rp), _p(ci), _p(v0), 0, 0, 0, _s(),
                              ctypes.byref(h)) == -7
    # null output handle
    assert lib.sptrsv_analyze(T.n, T.nnz, _p(rp), _p(ci), _p(v), 0, 0, 0, _s(), None) == -1
