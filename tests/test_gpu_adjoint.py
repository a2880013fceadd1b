"""Adjoint of x = T^{-1} b through torch.autograd (SpTRSVFunction): gradcheck
on a 4^3 ILU(0) factor, dense reference gradient and finite differences on
16^3, and the 96^3 ILU(0) factor against the oracle's adjoint."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpuhelp import dev, dev_tri, host, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_1710_04985_amd as sp
    return sp


@pytest.mark.parametrize("opts", [dict(algo=1), dict(algo=2, sync=0), dict(algo=2, sync=1)])
def test_gradcheck_ilu4(sp, opts):
    T = W.ilu0_lower((4, 4, 4))
    # perturb the unit diagonal so the diagonal's gradient is exercised too
    T.vals = T.vals * W.uniform_vector(T.nnz, 3, 0.8, 1.2)
    rp, ci, v = dev_tri(T)
    h = sp.Handle(rp, ci, v.clone()).configure(**opts)
    vals = v.clone().requires_grad_(True)
    b = dev(W.uniform_vector(T.n, 4)).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda vv, bb: sp.sptrsv(vv, bb, h), (vals, b),
                                    eps=1e-6, atol=1e-8, rtol=1e-6)


def test_dense_and_fd_16(sp):
    """Loss <w, x>; dense reference gradient (grad_b = T^{-T} w,
    grad_T = -grad_b x^T on the pattern) and central finite differences."""
    T, b_np, w_np = W.c5_ilu3d(side=16)
    rp, ci, v = dev_tri(T)
    h = sp.Handle(rp, ci, v.clone())
    vals = v.clone().requires_grad_(True)
    b = dev(b_np).requires_grad_(True)
    w = dev(w_np)
    x = sp.sptrsv(vals, b, h)
    (x * w).sum().backward()
    M = T.dense()
    xd = np.linalg.solve(M, b_np)
    gb = np.linalg.solve(M.T, w_np)
    rows = np.repeat(np.arange(T.n), np.diff(T.row_ptr))
    gv = -gb[rows] * xd[T.col_idx]
    assert relerr(host(x), xd) <= 1e-12
    assert relerr(host(b.grad), gb) <= 1e-10
    assert relerr(host(vals.grad), gv) <= 1e-10
    rng = np.random.Generator(np.random.PCG64(9))
    hstep = 1e-6
    an = host(vals.grad)
    ab = host(b.grad)
    for _ in range(3):
        dv = rng.uniform(-1, 1, T.nnz)
        db = rng.uniform(-1, 1, T.n)
        with torch.no_grad():
            lp = float((sp.sptrsv(v + hstep * dev(dv), dev(b_np + hstep * db), h) * w).sum())
            lm = float((sp.sptrsv(v - hstep * dev(dv), dev(b_np - hstep * db), h) * w).sum())
        fd = (lp - lm) / (2 * hstep)
        ref = an @ dv + ab @ db
        assert abs(fd - ref) <= 1e-6 * max(1.0, abs(ref))


@pytest.mark.parametrize("opts", [dict(algo=1), dict(algo=2, sync=0), dict(algo=2, sync=1)])
def test_ilu96_against_oracle(sp, opts):
    o = oracle.get()
    T, b_np, w_np = W.c5_ilu3d(side=96)
    rp, ci, v = dev_tri(T)
    h = sp.Handle(rp, ci, v.clone()).configure(**opts)
    vals = v.clone().requires_grad_(True)
    b = dev(b_np).requires_grad_(True)
    x = sp.sptrsv(vals, b, h)
    (x * dev(w_np)).sum().backward()
    h.status()
    xo, gbo, gvo = o.adjoint(T.row_ptr, T.col_idx, T.vals, b_np, w_np)
    assert relerr(host(x), xo) <= 1e-12
    assert relerr(host(b.grad), gbo) <= 1e-12
    assert relerr(host(vals.grad), gvo) <= 1e-12


def test_batched_grad(sp):
    o = oracle.get()
    tris = [W.ilu0_lower((s, s)) for s in (9, 14, 6)]
    devs = [dev_tri(t) for t in tris]
    bh = sp.BatchedHandle([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs])
    bs = [W.uniform_vector(t.n, i) for i, t in enumerate(tris)]
    ws = [W.uniform_vector(t.n, 10 + i) for i, t in enumerate(tris)]
    x = bh.solve(dev(np.concatenate(bs)))
    gb = bh.solve_t(dev(np.concatenate(ws)))
    gv = host(bh.grad_vals(gb, x))
    x, gb = host(x), host(gb)
    off = eoff = 0
    for t, b, w in zip(tris, bs, ws):
        xo, gbo, gvo = o.adjoint(t.row_ptr, t.col_idx, t.vals, b, w)
        assert relerr(x[off:off + t.n], xo) <= 1e-12
        assert relerr(gb[off:off + t.n], gbo) <= 1e-12
        assert relerr(gv[eoff:eoff + t.nnz], gvo) <= 1e-12
        off += t.n
        eoff += t.nnz


def test_chained_calls_share_one_handle(sp):
    """y = T2^{-1} (T1^{-1} b) with T1, T2 two value sets on ONE handle: the
    first call's backward runs after the second forward re-gathered other
    values, so it must gather its own again.  Dense reference gradients."""
    T = W.ilu0_lower((5, 5, 4))
    v1 = T.vals * W.uniform_vector(T.nnz, 21, 0.8, 1.2)
    v2 = T.vals * W.uniform_vector(T.nnz, 22, 0.7, 1.3)
    rp, ci, _ = dev_tri(T)
    h = sp.Handle(rp, ci, dev(v1))
    a1 = dev(v1).requires_grad_(True)
    a2 = dev(v2).requires_grad_(True)
    b_np = W.uniform_vector(T.n, 23)
    w_np = W.uniform_vector(T.n, 24)
    b = dev(b_np).requires_grad_(True)
    y = sp.sptrsv(a2, sp.sptrsv(a1, b, h), h)
    (y * dev(w_np)).sum().backward()
    rows = np.repeat(np.arange(T.n), np.diff(T.row_ptr))
    M1 = np.zeros((T.n, T.n))
    M2 = np.zeros((T.n, T.n))
    M1[rows, T.col_idx] = v1
    M2[rows, T.col_idx] = v2
    z = np.linalg.solve(M1, b_np)
    yd = np.linalg.solve(M2, z)
    g2 = np.linalg.solve(M2.T, w_np)            # d loss / d z
    g1 = np.linalg.solve(M1.T, g2)              # d loss / d b
    assert relerr(host(y), yd) <= 1e-12
    assert relerr(host(b.grad), g1) <= 1e-10
    assert relerr(host(a2.grad), -g2[rows] * yd[T.col_idx]) <= 1e-10
    assert relerr(host(a1.grad), -g1[rows] * z[T.col_idx]) <= 1e-10
