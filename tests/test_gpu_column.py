"""GPU parity of the column-wise solves (Sec. 3.2 sweep; Sec. 4.1 LEVC,
Sec. 4.2 SLFC) against the CPU oracle.

The updates pushed into a row arrive in an order fixed by timing, so the bar
is the floating-point tolerance (FP64 1e-12, FP32 1e-5 relative, inf-norm),
except where every partial sum is exact (diagonal matrix, integer prefix
sums): there the result is bit-exact whatever the order.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpuhelp import dev, dev_tri, host, relerr

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
LEVC, SLFC = 4, 5


@pytest.fixture(scope="module")
def sp():
    import paper_1710_04985_amd as sp
    assert torch.cuda.is_available()
    return sp


CASES = [("c1_lap2d_64", W.c1_lap2d_64()[0]),
         ("lap3d_20_L", W.laplacian_triangle((20, 20, 20))),
         ("lap3d_17x9x5_U", W.laplacian_triangle((17, 9, 5), upper=True)),
         ("powerlaw_50k", W.powerlaw_lower(50000, 21, window=5000)),
         ("ilu0_12", W.ilu0_lower((12, 12, 12))),
         ("rand_upper", W.random_triangle(300, 5, density=0.05, upper=True, shuffle_rows=True)),
         ("dense_rand_200_L", W.random_triangle(200, 8, density=0.9)),
         ("st27_12x11x10_U", W.stencil_triangle((12, 11, 10), 27, upper=True))]

SCHEDULES = [("levc", dict(algo=LEVC)), ("levc_g4", dict(algo=LEVC, group=4)),
             ("slfc", dict(algo=SLFC)), ("slfc_g1", dict(algo=SLFC, group=1)),
             ("slfc_g16_grid3", dict(algo=SLFC, group=16, grid=3)),
             ("slfc_xcd_grid16", dict(algo=SLFC, assign=2, grid=16)),
             ("slfc_epl1_wg256", dict(algo=SLFC, entries_per_lane=1, wg=256, grid=2))]


@pytest.mark.parametrize("sched,opts", SCHEDULES, ids=[s[0] for s in SCHEDULES])
@pytest.mark.parametrize("name,T", CASES, ids=[c[0] for c in CASES])
def test_column_solve_fp64(sp, name, T, sched, opts):
    print("column", name, sched, flush=True)
    o = oracle.get()
    b = W.uniform_vector(T.n, 11)
    h = sp.Handle(*dev_tri(T), uplo="U" if T.upper else "L").configure(**opts)
    x = host(h.solve(dev(b)))
    y = host(h.solve_t(dev(b)))
    h.status()
    assert relerr(x, o.solve(T.row_ptr, T.col_idx, T.vals, b, T.upper)) <= TOL64
    assert relerr(y, o.solve_transpose(T.row_ptr, T.col_idx, T.vals, b, T.upper)) <= TOL64


@pytest.mark.parametrize("algo", [LEVC, SLFC])
def test_column_solve_fp32(sp, algo):
    o = oracle.get()
    T = W.powerlaw_lower(40000, 5, window=4000)
    v32 = T.vals.astype(np.float32)
    b32 = W.uniform_vector(T.n, 6).astype(np.float32)
    h = sp.Handle(*dev_tri(T, torch.float32)).configure(algo=algo)
    x = host(h.solve(dev(b32)))
    h.status()
    ref = o.solve(T.row_ptr, T.col_idx, v32.astype(np.float64), b32.astype(np.float64))
    assert relerr(x, ref) <= TOL32


@pytest.mark.parametrize("algo", [LEVC, SLFC])
def test_column_exact_cases(sp, algo):
    """Diagonal: no updates, x = b * (1/d); chain I - S with integer b: every
    partial sum is an integer below 2^53, so the order cannot matter."""
    d = W.uniform_vector(5000, 1, 0.5, 3.0)
    b = W.uniform_vector(5000, 2)
    h = sp.Handle(*dev_tri(W.diagonal_matrix(d))).configure(algo=algo)
    assert np.array_equal(host(h.solve(dev(b))), b * (1.0 / d))
    n = 100000 if algo == SLFC else 5000
    rng = np.random.Generator(np.random.PCG64(4))
    bi = rng.integers(-1000, 1000, n).astype(np.float64)
    for upper in (False, True):
        P = W.bidiagonal_fast(n, 1.0, 1.0, upper=upper)
        h = sp.Handle(*dev_tri(P), uplo="U" if upper else "L").configure(algo=algo)
        want = np.cumsum(bi[::-1])[::-1] if upper else np.cumsum(bi)
        assert np.array_equal(host(h.solve(dev(bi))), want)
        # the transposed chain runs the other way
        want_t = np.cumsum(bi) if upper else np.cumsum(bi[::-1])[::-1]
        assert np.array_equal(host(h.solve_t(dev(bi))), want_t)
        h.status()


@pytest.mark.parametrize("algo", [LEVC, SLFC])
def test_column_in_place_unit_and_update(sp, algo):
    o = oracle.get()
    T = W.ilu0_lower((11, 10, 9))
    b = W.uniform_vector(T.n, 5)
    h = sp.Handle(*dev_tri(T), unit_diag=True).configure(algo=algo)
    x = dev(b)
    h.solve(x, out=x)
    h.status()
    assert relerr(host(x), o.solve(T.row_ptr, T.col_idx, T.vals, b, False, True)) <= TOL64
    # new values, same pattern: the push copy is re-gathered
    v2 = T.vals * 0.5
    h.update_values(dev(v2))
    x = host(h.solve(dev(b)))
    y = host(h.solve_t(dev(b)))
    h.status()
    assert relerr(x, o.solve(T.row_ptr, T.col_idx, v2, b, False, True)) <= TOL64
    assert relerr(y, o.solve_transpose(T.row_ptr, T.col_idx, v2, b, False, True)) <= TOL64


def test_column_multi_rhs_uses_row_solve(sp):
    o = oracle.get()
    T = W.laplacian_triangle((14, 13, 12), upper=True)
    B = np.stack([W.uniform_vector(T.n, 20 + r) for r in range(5)])
    h = sp.Handle(*dev_tri(T), uplo="U").configure(algo=SLFC)
    X = host(h.solve_multi(dev(B)))
    h.status()
    ref = o.solve_multi(T.row_ptr, T.col_idx, T.vals, B.T, True)
    assert relerr(X.T, ref) <= TOL64


def test_column_watchdog_and_recovery(sp):
    n = 20000
    P = W.bidiagonal_fast(n, 1.0, 1.0)
    b = np.ones(n)
    h = sp.Handle(*dev_tri(P)).configure(algo=SLFC, spin_limit=1)
    h.solve(dev(b))
    with pytest.raises(sp.SpTRSVError) as e:
        h.status()
    assert e.value.status == -10
    h.set_option("spin_limit", 1 << 22)
    x = host(h.solve(dev(b)))
    h.status()
    assert np.array_equal(x, np.arange(1, n + 1, dtype=np.float64))


@pytest.mark.parametrize("algo", [LEVC, SLFC])
def test_column_graph_replay(sp, algo):
    o = oracle.get()
    T = W.laplacian_triangle((24, 23, 22))
    bh = W.uniform_vector(T.n, 2)
    ref = o.solve(T.row_ptr, T.col_idx, T.vals, bh)
    ref_t = o.solve_transpose(T.row_ptr, T.col_idx, T.vals, bh)
    h = sp.Handle(*dev_tri(T)).configure(algo=algo)
    s = torch.cuda.Stream()
    b = dev(bh)
    x = torch.empty_like(b)
    with torch.cuda.stream(s):
        g = h.capture(b, x, stream=s)
        gt = h.capture(b, x, transpose=True, stream=s)
        for rep in range(4):
            x.zero_()
            g.launch(s)
            s.synchronize()
            assert relerr(host(x), ref) <= TOL64, rep
            h.solve(b * 2.0)                   # eager work between replays
            s.synchronize()
            gt.launch(s)
            s.synchronize()
            assert relerr(host(x), ref_t) <= TOL64, rep
    h.status()


def test_column_tune(sp):
    o = oracle.get()
    T = W.laplacian_triangle((30, 30, 30))
    h = sp.Handle(*dev_tri(T)).configure(algo=SLFC)
    b = dev(W.uniform_vector(T.n, 3))
    info = h.tune(b)
    assert info["algo"] == SLFC
    x = host(h.solve(b))
    h.status()
    assert relerr(x, o.solve(T.row_ptr, T.col_idx, T.vals, host(b))) <= TOL64
