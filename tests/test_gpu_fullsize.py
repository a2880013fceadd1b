"""Full-size parity in the launch configurations the benchmark times: every
workload at its real size, schedules chosen by the autotuner, against the
FP64 oracle (relative inf-norm error <= 1e-12; FP32 <= 1e-5 against the
oracle on the up-cast FP32 data), and every GPU result held to the
componentwise backward-error bound of substitution (scale-free: a small
component cannot hide behind the norm).  The 96^3 ILU(0) adjoint is covered
at full size in test_gpu_adjoint.py."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpuhelp import backward_error_ok, dev, dev_tri, host, relerr

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def sp():
    import paper_1710_04985_amd as sp
    assert torch.cuda.is_available()
    return sp


def _tuned_pair(sp, T, b):
    """Self-scheduled handle tuned among self-scheduled schedules and a
    level-scheduled one tuned among its own, as the benchmark does."""
    uplo = "U" if T.upper else "L"
    hs = sp.Handle(*dev_tri(T), uplo=uplo)
    hs.set_option("algo", sp.ALGO_SELF)
    hs.tune(b)
    hl = sp.Handle(*dev_tri(T), uplo=uplo)
    hl.set_option("algo", sp.ALGO_LEVEL)
    hl.tune(b)
    return hs, hl


def test_c1_lap2d_64(sp):
    print("full size: C1", flush=True)
    T, xs, b = W.c1_lap2d_64()
    xo = oracle.get().solve(T.row_ptr, T.col_idx, T.vals, b)
    hs, hl = _tuned_pair(sp, T, dev(b))
    for h in (hs, hl):
        x = host(h.solve(dev(b)))
        h.status()
        assert relerr(x, xo) <= TOL64
        assert relerr(x, xs) <= 1e-10          # the planted solution (well conditioned)
        assert backward_error_ok(T, b, x)[0]


def test_c2_lap3d_128_lower_then_upper(sp):
    """The benchmark step: lower solve, then the upper solve of its result."""
    print("full size: C2 lower then upper", flush=True)
    o = oracle.get()
    TL, xsL, bL = W.c2_lap3d(upper=False)
    TU = W.laplacian_triangle((128, 128, 128), upper=True, diag=6.0)
    y1o = o.solve(TL.row_ptr, TL.col_idx, TL.vals, bL, False)
    y2o = o.solve(TU.row_ptr, TU.col_idx, TU.vals, y1o, True)
    b = dev(bL)
    hsL, hlL = _tuned_pair(sp, TL, b)
    hsU, hlU = _tuned_pair(sp, TU, b)
    for hL, hU in ((hsL, hsU), (hlL, hlU)):
        y1 = hL.solve(b)
        y2 = hU.solve(y1)
        hL.status()
        hU.status()
        assert relerr(host(y1), y1o) <= TOL64
        assert relerr(host(y2), y2o) <= TOL64
        assert backward_error_ok(TL, bL, host(y1))[0]
        assert backward_error_ok(TU, host(y1), host(y2))[0]
    # the transposed solves of the same handles
    g = W.uniform_vector(TL.n, 8)
    assert relerr(host(hsL.solve_t(dev(g))),
                  o.solve_transpose(TL.row_ptr, TL.col_idx, TL.vals, g, False)) <= TOL64
    hsL.status()


def test_c3_powerlaw_fp64_and_fp32(sp):
    print("full size: C3 power-law", flush=True)
    o = oracle.get()
    T, xs, b = W.c3_powerlaw()
    xo = o.solve(T.row_ptr, T.col_idx, T.vals, b)
    hs, hl = _tuned_pair(sp, T, dev(b))
    for h in (hs, hl):
        x = host(h.solve(dev(b)))
        h.status()
        assert relerr(x, xo) <= TOL64
        assert backward_error_ok(T, b, x)[0]
    v32 = T.vals.astype(np.float32)
    b32 = b.astype(np.float32)
    xo32 = o.solve(T.row_ptr, T.col_idx, v32.astype(np.float64), b32.astype(np.float64))
    h32 = sp.Handle(*dev_tri(T, torch.float32))
    h32.set_option("algo", sp.ALGO_SELF)
    h32.tune(dev(b32))
    x32 = host(h32.solve(dev(b32)))
    h32.status()
    assert relerr(x32, xo32) <= TOL32
    T32 = W.Triangle(T.n, T.row_ptr, T.col_idx, v32.astype(np.float64))
    assert backward_error_ok(T32, b32, x32, unit_roundoff=2.0 ** -24)[0]


def test_c4a_batched_256_graph(sp):
    """256 uneven ILU(0) factors, one launch, replayed from a HIP graph."""
    print("full size: C4a batched", flush=True)
    o = oracle.get()
    tris, xs, bs = W.c4a_batch()
    devs = [dev_tri(t) for t in tris]
    xo = np.concatenate([o.solve(t.row_ptr, t.col_idx, t.vals, bb) for t, bb in zip(tris, bs)])
    Tcat = W.concat_block_diagonal(tris)
    bd = dev(np.concatenate(bs))
    x = torch.empty_like(bd)
    for algo in (sp.ALGO_SELF, sp.ALGO_LEVEL, sp.ALGO_BLOCK):
        h = sp.BatchedHandle([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs])
        h.set_option("algo", algo)
        if algo != sp.ALGO_BLOCK:
            h.tune(bd, x)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            g = h.capture(bd, x, stream=s)
            for rep in range(3):
                x.zero_()
                g.launch(s)
                s.synchronize()
                assert relerr(host(x), xo) <= TOL64, (algo, rep)
            assert backward_error_ok(Tcat, np.concatenate(bs), host(x))[0], algo
            g.close()
        h.status()


def test_c4b_16_rhs(sp):
    print("full size: C4b 16 RHS", flush=True)
    o = oracle.get()
    T, X, B = W.c4b_multi(nrhs=16)
    Bd = dev(np.ascontiguousarray(B.T))
    h = sp.Handle(*dev_tri(T))
    h.set_option("algo", sp.ALGO_SELF)
    h.tune_multi(Bd)
    Xd = host(h.solve_multi(Bd))
    h.status()
    Xo = o.solve_multi(T.row_ptr, T.col_idx, T.vals, B)
    assert relerr(Xd.T, Xo) <= TOL64
    for q in (0, 7, 15):
        assert backward_error_ok(T, B[:, q], Xd[q])[0], q


def test_table2_deepest_grid_9pt(sp):
    """The deepest grid of the paper's Table 2: the 9-point operator on
    64 x 16384 (n = 2^20), lower then upper (32,830 levels each), self- and
    level-scheduled."""
    print("full size: Table 2 64x16384 9-point", flush=True)
    o = oracle.get()
    L = W.stencil_triangle((64, 16384), 9)
    U = W.stencil_triangle((64, 16384), 9, upper=True)
    b = W.uniform_vector(L.n, 7)
    y1o = o.solve(L.row_ptr, L.col_idx, L.vals, b, False)
    y2o = o.solve(U.row_ptr, U.col_idx, U.vals, y1o, True)
    bd = dev(b)
    hsL, hlL = _tuned_pair(sp, L, bd)
    hsU, hlU = _tuned_pair(sp, U, bd)
    assert hsL.info()["nlev"] == 32830 and hsU.info()["nlev"] == 32830
    for hL, hU in ((hsL, hsU), (hlL, hlU)):
        y1 = hL.solve(bd)
        y2 = hU.solve(y1)
        hL.status()
        hU.status()
        assert relerr(host(y1), y1o) <= TOL64
        assert relerr(host(y2), y2o) <= TOL64
        assert backward_error_ok(L, b, host(y1))[0]
        assert backward_error_ok(U, host(y1), host(y2))[0]
