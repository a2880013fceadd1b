"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bars: analysis (levels, level sets, dependency counts) bit-exact; FP64
solves within 1e-12 relative (inf-norm) of the FP64 oracle, FP32 within 1e-5
of the FP64 oracle run on the FP32 data; exactly representable cases
bit-exact; level- and self-scheduled solves bit-identical at equal lanes per
row (a race would show up as a difference).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpuhelp import DEV, bits_equal, dev, dev_tri, host, relerr

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def sp():
    import paper_1710_04985_amd as sp
    assert torch.cuda.is_available()
    return sp


def _small_cases():
    cases = [("c1_lap2d_64", W.c1_lap2d_64()[0]),
             ("lap3d_20_L", W.laplacian_triangle((20, 20, 20))),
             ("lap3d_20_U", W.laplacian_triangle((20, 20, 20), upper=True)),
             ("lap3d_17x9x5_U", W.laplacian_triangle((17, 9, 5), upper=True)),
             ("powerlaw_50k", W.powerlaw_lower(50000, 21, window=5000)),
             ("ilu0_12", W.ilu0_lower((12, 12, 12))),
             ("rand_upper", W.random_triangle(300, 5, density=0.05, upper=True, shuffle_rows=True)),
             ("rand_lower", W.random_triangle(257, 6, density=0.08, shuffle_rows=True)),
             ("st9_30x20_L", W.stencil_triangle((30, 20), 9)),
             ("st27_12x11x10_U", W.stencil_triangle((12, 11, 10), 27, upper=True))]
    return cases


CASES = _small_cases()
SCHEDULES = [("level", dict(algo=1)), ("self_value", dict(algo=2, sync=0)),
             ("block", dict(algo=3)), ("block_wg_ignored", dict(algo=3, group=4)),
             ("block_streamed", dict(algo=3, block_resident=0)),
             ("self_ticket", dict(algo=2, sync=0, assign=1)),
             ("self_static_g4_grid3", dict(algo=2, sync=0, assign=0, group=4, grid=3)),
             ("self_static_wg256", dict(algo=2, sync=0, assign=0, wg=256, grid=2)),
             ("self_xcd_grid16", dict(algo=2, sync=0, assign=2, grid=16)),
             ("self_xcd_grid5", dict(algo=2, sync=0, assign=2, grid=5)),
             ("self_flag", dict(algo=2, sync=1)), ("self_value_g1", dict(algo=2, group=1)),
             ("self_value_g8", dict(algo=2, group=8)), ("level_g64", dict(algo=1, group=64)),
             ("self_flag_g16", dict(algo=2, sync=1, group=16)),
             ("self_value_epl1", dict(algo=2, entries_per_lane=1)),
             ("self_value_rpl1_grid8", dict(algo=2, rows_per_lane=1, grid=8)),
             ("level_rpl2", dict(algo=1, rows_per_lane=2, group=1)),
             ("self_flag_rpl3_wg256", dict(algo=2, sync=1, rows_per_lane=3, wg=256, grid=4)),
             ("self_value_wg256_grid1", dict(algo=2, wg=256, grid=1)),
             ("self_static_poll0", dict(algo=2, sync=0, assign=0, poll=0)),
             ("self_xcd_poll0_grid16", dict(algo=2, sync=0, assign=2, grid=16, poll=0)),
             ("self_ticket_poll0", dict(algo=2, sync=0, assign=1, poll=0)),
             ("self_static_stride2", dict(algo=2, sync=0, assign=0, xp_stride=2)),
             ("self_xcd_stride2_poll0", dict(algo=2, sync=0, assign=2, grid=16, poll=0,
                                             xp_stride=2)),
             ("self_static_stride8", dict(algo=2, sync=0, assign=0, xp_stride=8)),
             ("self_xcd_stride16", dict(algo=2, sync=0, assign=2, grid=16, xp_stride=16))]


@pytest.mark.parametrize("name,T", CASES, ids=[c[0] for c in CASES])
def test_analysis_export_bit_exact(sp, name, T):
    o = oracle.get()
    h = sp.Handle(*dev_tri(T), uplo="U" if T.upper else "L", unit_diag=T.unit_diag)
    level, ilev, jlev, dep = h.export_analysis()
    lv, nlev, il, jl, dc = o.analyze(T.row_ptr, T.col_idx, T.upper)
    assert np.array_equal(level, lv) and np.array_equal(ilev, il)
    assert np.array_equal(jlev, jl) and np.array_equal(dep, dc)
    assert h.info()["nlev"] == nlev
    # analysis of T^T
    rT, cT, _ = o.transpose(T.row_ptr, T.col_idx)
    lvT, nlevT, ilT, jlT, dcT = o.analyze(rT, cT, not T.upper)
    level, ilev, jlev, dep = h.export_analysis(transpose=True)
    assert np.array_equal(level, lvT) and np.array_equal(ilev, ilT)
    assert np.array_equal(jlev, jlT) and np.array_equal(dep, dcT)
    assert nlevT == nlev


@pytest.mark.parametrize("sched,opts", SCHEDULES, ids=[s[0] for s in SCHEDULES])
@pytest.mark.parametrize("name,T", CASES, ids=[c[0] for c in CASES])
def test_solve_fp64(sp, name, T, sched, opts):
    o = oracle.get()
    h = sp.Handle(*dev_tri(T), uplo="U" if T.upper else "L").configure(**opts)
    b = W.uniform_vector(T.n, 7)
    xo = o.solve(T.row_ptr, T.col_idx, T.vals, b, T.upper)
    x = h.solve(dev(b))
    h.status()
    assert relerr(host(x), xo) <= TOL64
    # transposed solve
    g = W.uniform_vector(T.n, 8)
    yo = o.solve_transpose(T.row_ptr, T.col_idx, T.vals, g, T.upper)
    y = h.solve_t(dev(g))
    h.status()
    assert relerr(host(y), yo) <= TOL64


@pytest.mark.parametrize("name,T", CASES[:5], ids=[c[0] for c in CASES[:5]])
def test_solve_fp32(sp, name, T):
    o = oracle.get()
    v32 = T.vals.astype(np.float32)
    b32 = W.uniform_vector(T.n, 9).astype(np.float32)
    xo = o.solve(T.row_ptr, T.col_idx, v32.astype(np.float64), b32.astype(np.float64), T.upper)
    ref = None
    for opts in (dict(algo=1), dict(algo=2, sync=0), dict(algo=2, sync=1),
                 dict(algo=2, sync=0, xp_stride=2), dict(algo=2, assign=2, poll=0, xp_stride=2),
                 dict(algo=2, sync=0, xp_stride=16), dict(algo=3), dict(algo=3, block_resident=0)):
        h = sp.Handle(dev(T.row_ptr), dev(T.col_idx), dev(v32),
                      uplo="U" if T.upper else "L").configure(**opts)
        x = h.solve(dev(b32))
        h.status()
        assert x.dtype == torch.float32
        assert relerr(host(x), xo) <= TOL32, opts
        if opts.get("algo") == 2 and opts.get("sync") == 0 and "assign" not in opts:
            # 8-byte slots change where values live, not how they are computed
            if ref is None:
                ref = x
            else:
                assert bits_equal(x, ref)


@pytest.mark.parametrize("group,rpl", [(1, 1), (1, 4), (0, 4), (4, 1), (16, 1), (64, 1)])
@pytest.mark.parametrize("name,T", [CASES[1], CASES[4], CASES[6]], ids=[CASES[1][0], CASES[4][0], CASES[6][0]])
def test_level_equals_self_bitwise(sp, name, T, group, rpl):
    """Same per-row arithmetic under every schedule: results must be
    bit-identical, on every one of repeated solves."""
    b = dev(W.uniform_vector(T.n, 11))
    hl = sp.Handle(*dev_tri(T), uplo="U" if T.upper else "L").configure(algo=1, group=group,
                                                                        rows_per_lane=rpl)
    ref = hl.solve(b)
    if group == 1:
        hb = sp.Handle(*dev_tri(T), uplo="U" if T.upper else "L").configure(algo=3)
        for _ in range(5):
            assert bits_equal(hb.solve(b), ref)
    for sync, assign, poll, stride in ((0, 0, 1, 1), (0, 1, 1, 1), (1, 1, 1, 1), (0, 2, 1, 1),
                                       (0, 0, 0, 1), (0, 1, 0, 1), (0, 0, 1, 2), (0, 2, 0, 2),
                                       (0, 0, 1, 4), (0, 2, 1, 8), (0, 0, 0, 16)):
        if assign in (0, 2) and rpl != 1:
            continue                  # static assignment keeps one row per lane
        hs = sp.Handle(*dev_tri(T), uplo="U" if T.upper else "L").configure(
            algo=2, group=group, sync=sync, rows_per_lane=rpl, assign=assign, poll=poll,
            xp_stride=stride)
        for _ in range(20):
            assert bits_equal(hs.solve(b), ref)
        hs.status()


@pytest.mark.parametrize("opts", [dict(algo=2, assign=0), dict(algo=2, assign=2, poll=0),
                                  dict(algo=2, assign=1), dict(algo=2, sync=1), dict(algo=3),
                                  dict(algo=5)])
def test_alternating_right_hand_sides(sp, opts):
    """Consecutive solves on one handle with different b: every solve must
    produce its own answer (a value left over from the previous solve would
    be read as published if readiness ever leaked across solves)."""
    T = W.laplacian_triangle((24, 22, 20))
    hl = sp.Handle(*dev_tri(T)).configure(algo=1)
    bs = [dev(W.uniform_vector(T.n, 40 + k)) for k in range(3)]
    refs = [hl.solve(b) for b in bs]
    h = sp.Handle(*dev_tri(T)).configure(**opts)
    for it in range(12):
        k = it % 3
        x = h.solve(bs[k])
        if opts.get("algo") == 5:
            assert relerr(host(x), host(refs[k])) <= TOL64, it
        else:
            assert bits_equal(x, refs[k]), it
    h.status()


@pytest.mark.parametrize("opts", [dict(algo=1), dict(algo=2, sync=0), dict(algo=2, sync=1)])
def test_in_place(sp, opts):
    o = oracle.get()
    T = W.laplacian_triangle((15, 14, 13))
    b = W.uniform_vector(T.n, 3)
    h = sp.Handle(*dev_tri(T)).configure(**opts)
    x = dev(b)
    h.solve(x, out=x)
    y = dev(b)
    h.solve_t(y, out=y)
    h.status()
    assert relerr(host(x), o.solve(T.row_ptr, T.col_idx, T.vals, b)) <= TOL64
    assert relerr(host(y), o.solve_transpose(T.row_ptr, T.col_idx, T.vals, b)) <= TOL64


@pytest.mark.parametrize("opts", [dict(algo=1), dict(algo=2, sync=0), dict(algo=2, sync=1),
                                  dict(algo=2, sync=0, assign=1), dict(algo=3)])
def test_exact_cases(sp, opts):
    """Diagonal: x = b * (1/d), the kernels' rounding (within 1.5 ulp of
    b/d); chain I - S (nlev = n): prefix sums of integers; bidiagonal (2, -1)
    with b = e_0: x_i = 2^-(i+1).  Bit-exact."""
    d = W.uniform_vector(5000, 1, 0.5, 3.0)
    D = W.diagonal_matrix(d)
    b = W.uniform_vector(5000, 2)
    h = sp.Handle(*dev_tri(D)).configure(**opts)
    x = host(h.solve(dev(b)))
    assert np.array_equal(x, b * (1.0 / d))
    assert np.all(np.abs(x - b / d) <= 1.5 * np.spacing(np.abs(b / d)))
    n = 200000 if opts["algo"] == 2 else 20000      # level-scheduled: one launch per row
    rng = np.random.Generator(np.random.PCG64(4))
    bi = rng.integers(-1000, 1000, n).astype(np.float64)
    for upper in (False, True):
        P = W.bidiagonal_fast(n, 1.0, 1.0, upper=upper)
        h = sp.Handle(*dev_tri(P), uplo="U" if upper else "L").configure(**opts)
        want = np.cumsum(bi[::-1])[::-1] if upper else np.cumsum(bi)
        assert np.array_equal(host(h.solve(dev(bi))), want)
        h.status()
    B = W.bidiagonal_fast(600, 2.0, 1.0)
    e = np.zeros(600)
    e[0] = 1.0
    h = sp.Handle(*dev_tri(B)).configure(**opts)
    x = host(h.solve(dev(e)))
    assert np.array_equal(x, 2.0 ** -(np.arange(600) + 1.0))


def test_unit_diag(sp):
    o = oracle.get()
    T = W.ilu0_lower((11, 10, 9))          # stored unit diagonal
    b = W.uniform_vector(T.n, 5)
    xo = o.solve(T.row_ptr, T.col_idx, T.vals, b, False, True)
    for opts in (dict(algo=1), dict(algo=2, sync=0), dict(algo=2, sync=1), dict(algo=3),
                 dict(algo=3, block_resident=0)):
        h = sp.Handle(*dev_tri(T), unit_diag=True).configure(**opts)
        assert relerr(host(h.solve(dev(b))), xo) <= TOL64
    # diagonal entries absent altogether
    rows = np.repeat(np.arange(T.n), np.diff(T.row_ptr))
    keep = T.col_idx != rows
    rp = np.zeros(T.n + 1, np.int32)
    rp[1:] = np.cumsum(np.bincount(rows[keep], minlength=T.n))
    h = sp.Handle(dev(rp), dev(T.col_idx[keep]), dev(T.vals[keep]), unit_diag=True)
    assert relerr(host(h.solve(dev(b))), xo) <= TOL64
    # a 2-D unit-diagonal factor narrow enough for the whole-system-in-LDS kernel
    T2 = W.ilu0_lower((40, 30))
    b2 = W.uniform_vector(T2.n, 6)
    xo2 = o.solve(T2.row_ptr, T2.col_idx, T2.vals, b2, False, True)
    xs = [sp.Handle(*dev_tri(T2), unit_diag=True).configure(algo=3, block_resident=r).solve(dev(b2))
          for r in (1, 0)]
    assert bits_equal(xs[0], xs[1])
    assert relerr(host(xs[0]), xo2) <= TOL64


@pytest.mark.parametrize("nrhs", [1, 3, 16, 70])
@pytest.mark.parametrize("opts", [dict(algo=1), dict(algo=2), dict(algo=2, assign=1),
                                  dict(algo=2, grid=3), dict(algo=2, assign=2, grid=32),
                                  dict(algo=2, multi_rows=1), dict(algo=2, multi_rows=2, grid=5),
                                  dict(algo=2, multi_rows=4, assign=2, grid=16)])
def test_multi_rhs(sp, nrhs, opts):
    o = oracle.get()
    T = W.laplacian_triangle((14, 13, 12), upper=True)
    F = np.stack([W.uniform_vector(T.n, 100 + r) for r in range(nrhs)], 0)     # (nrhs, n)
    h = sp.Handle(*dev_tri(T), uplo="U").configure(group=1, **opts)
    X = host(h.solve_multi(dev(F)))
    Xt = host(h.solve_multi(dev(F), transpose=True))
    h.status()
    Xo = o.solve_multi(T.row_ptr, T.col_idx, T.vals, F.T, True)
    for r in range(nrhs):
        assert relerr(X[r], Xo[:, r]) <= TOL64
        assert relerr(Xt[r], o.solve_transpose(T.row_ptr, T.col_idx, T.vals, F[r], True)) <= TOL64
    # every column equals the single right-hand-side solve, bit for bit
    for r in (0, nrhs - 1):
        assert bits_equal(X[r], host(h.solve(dev(F[r]))))
    # in place
    B = dev(F)
    h.solve_multi(B, out=B)
    assert bits_equal(host(B), X)
    # the multi-RHS tuner's schedule gives the same columns
    if nrhs >= 2:
        h.tune_multi(dev(F))
        X2 = host(h.solve_multi(dev(F)))
        h.status()
        assert bits_equal(X2, X)


@pytest.mark.parametrize("nrhs", [2, 5, 9])
@pytest.mark.parametrize("assign", [0, 1, 2])
def test_multi_rhs_strided(sp, nrhs, assign):
    """Column stride ld > n (row-slices of a wider buffer): the same bits as
    the contiguous solve, nothing written outside the columns; power-law rows
    long enough for several entry batches; FP32 within tolerance."""
    o = oracle.get()
    T = W.powerlaw_lower(30000, 13, window=3000)
    F = np.stack([W.uniform_vector(T.n, 300 + r) for r in range(nrhs)], 0)
    h = sp.Handle(*dev_tri(T)).configure(algo=2, assign=assign, grid=40)
    X = host(h.solve_multi(dev(F)))
    h.status()
    assert relerr(X.T, o.solve_multi(T.row_ptr, T.col_idx, T.vals, F.T)) <= TOL64
    wide = torch.zeros(nrhs, T.n + 7, dtype=torch.float64, device="cuda")
    wide[:, :T.n] = dev(F)
    Xw = torch.zeros_like(wide)
    h.solve_multi(wide[:, :T.n], out=Xw[:, :T.n])
    h.status()
    assert bits_equal(host(Xw[:, :T.n]), X)
    assert not host(Xw[:, T.n:]).any()
    # a strided result allocated by the binding
    Xs = h.solve_multi(wide[:, :T.n])
    assert Xs.stride() == (T.n + 7, 1)
    assert bits_equal(host(Xs), X)
    with pytest.raises(ValueError):
        h.solve_multi(wide[:, :T.n], out=torch.empty(nrhs, T.n, dtype=torch.float64, device="cuda"))
    v32 = T.vals.astype(np.float32)
    F32 = F.astype(np.float32)
    h32 = sp.Handle(*dev_tri(T, torch.float32)).configure(algo=2, assign=assign)
    X32 = host(h32.solve_multi(dev(F32)))
    h32.status()
    ref = o.solve_multi(T.row_ptr, T.col_idx, v32.astype(np.float64), F32.T.astype(np.float64))
    assert relerr(X32.T, ref) <= TOL32


def test_multi_rhs_long_rows_by_columns(sp):
    """Rows longer than 64 entries with the default lane rule: the columns
    are solved one after another by the single-RHS schedule, each equal to
    sptrsv_solve on it bit for bit; tune_multi leaves it.  T^T of this
    triangle has short rows (column counts), so the transposed solve takes
    the multi-RHS kernel: each column equals the one-lane-per-row solve_t."""
    o = oracle.get()
    T = W.powerlaw_lower(30000, 19, window=3000)
    assert np.diff(T.row_ptr).max() > 65
    F = np.stack([W.uniform_vector(T.n, 700 + r) for r in range(5)], 0)
    h = sp.Handle(*dev_tri(T))
    X = h.solve_multi(dev(F))
    Xt = h.solve_multi(dev(F), transpose=True)
    h.tune_multi(dev(F))
    X2 = h.solve_multi(dev(F))
    h.status()
    h1 = sp.Handle(*dev_tri(T)).configure(group=1)
    for r in range(5):
        assert bits_equal(X[r], h.solve(dev(F[r])))
        assert bits_equal(Xt[r], h1.solve_t(dev(F[r])))
    assert bits_equal(X2, X)
    assert relerr(host(X).T, o.solve_multi(T.row_ptr, T.col_idx, T.vals, F.T)) <= TOL64
    for r in (0, 4):
        assert relerr(host(Xt[r]), o.solve_transpose(T.row_ptr, T.col_idx, T.vals, F[r])) <= TOL64


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("opts", [dict(), dict(assign=2), dict(assign=0, grid=200),
                                  dict(assign=2, grid=512, xp_stride=1),
                                  dict(assign=2, grid=64, wg=256)])
def test_multi_rhs_long_rows_one_launch(sp, opts, dtype):
    """Rows longer than 64 entries, static schedule: all columns in one launch
    of the one-RHS kernel over a column-batched chunk table, with a leading
    dimension larger than n; every column equals sptrsv_solve on it bit for
    bit, the padding between columns is untouched, and the transposed solve
    of a pattern whose transpose has the long rows takes the same path."""
    T = W.powerlaw_lower(30000, 23, window=3000).astype_vals(dtype)
    assert np.diff(T.row_ptr).max() > 65
    nrhs, ld = 16, T.n + 37
    F = np.zeros((nrhs, ld), dtype)
    for r in range(nrhs):
        F[r, :T.n] = W.uniform_vector(T.n, 900 + r)
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    h = sp.Handle(*dev_tri(T, tdt)).configure(**opts)
    Fd = dev(F)
    Xd = torch.full_like(Fd, 7.0)
    h.solve_multi(Fd[:, :T.n], out=Xd[:, :T.n])
    h.status()
    X = host(Xd)
    for r in range(nrhs):
        assert bits_equal(X[r, :T.n], h.solve(dev(F[r, :T.n]))), r
        assert np.all(X[r, T.n:] == 7.0)
    # T^T with long rows: the upper triangle whose transpose is T
    S = T.scipy().T.tocsr()
    U = W.Triangle(T.n, S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data.astype(dtype),
                   upper=True)
    hu = sp.Handle(*dev_tri(U, tdt), uplo="U").configure(**opts)
    Xt = host(hu.solve_multi(dev(F[:, :T.n].copy()), transpose=True))
    hu.status()
    for r in (0, 7, 15):
        assert bits_equal(Xt[r], hu.solve_t(dev(F[r, :T.n].copy()))), r
    o = oracle.get()
    if dtype == np.float64:
        ref = o.solve_multi(T.row_ptr, T.col_idx, T.vals, F[:, :T.n].T)
        assert relerr(X[:, :T.n].T, ref) <= TOL64


@pytest.mark.parametrize("nrhs", [2, 6, 16, 33])
def test_multi_rows_per_lane_group(sp, nrhs):
    """Rows per lane group of the static multi-RHS kernel (1, 2, 4): the same
    bits for every choice and grid, and every column equal to the one-lane
    single-RHS solve; power-law rows long enough for several entry batches."""
    o = oracle.get()
    T = W.powerlaw_lower(40000, 17, window=4000)
    F = np.stack([W.uniform_vector(T.n, 500 + r) for r in range(nrhs)], 0)
    h = sp.Handle(*dev_tri(T)).configure(algo=2, group=1)
    ref = None
    for mr, grid, assign in ((1, 0, 0), (2, 7, 0), (4, 0, 2), (4, 64, 0), (0, 3, 2)):
        h.configure(multi_rows=mr, grid=grid, assign=assign)
        X = host(h.solve_multi(dev(F)))
        h.status()
        if ref is None:
            ref = X
            assert relerr(X.T, o.solve_multi(T.row_ptr, T.col_idx, T.vals, F.T)) <= TOL64
        assert bits_equal(X, ref), (mr, grid, assign)
    for r in (0, nrhs // 2, nrhs - 1):
        assert bits_equal(ref[r], host(h.solve(dev(F[r]))))


@pytest.mark.parametrize("name,T", [CASES[4], CASES[1], CASES[6]],
                         ids=[CASES[4][0], CASES[1][0], CASES[6][0]])
def test_tuned_result_is_reproducible(sp, name, T):
    """The autotuner varies only schedule dimensions that keep each row's
    summation order (its lanes stay as the options set them), so a tuned
    solve equals the untuned self-scheduled solve bit for bit, whichever
    candidate timing picks (rows up to 2,000 entries on the power-law case)."""
    b = dev(W.uniform_vector(T.n, 17))
    uplo = "U" if T.upper else "L"
    ref = sp.Handle(*dev_tri(T), uplo=uplo).configure(algo=2).solve(b)
    for algo in (0, 2):
        h = sp.Handle(*dev_tri(T), uplo=uplo).configure(algo=algo)
        x = torch.empty_like(b)
        h.tune(b, x)
        assert bits_equal(h.solve(b), ref), h.info()
        h.status()


def test_two_streams_are_serialized(sp):
    """Solves of one handle issued on two streams without any ordering by the
    caller: the library makes each stream wait for the handle's previous
    solve, so neither races on the shared scratch; with a value update in
    between on a third stream."""
    o = oracle.get()
    T = W.laplacian_triangle((40, 40, 40))
    bs = [W.uniform_vector(T.n, 60 + k) for k in range(4)]
    h = sp.Handle(*dev_tri(T)).configure(algo=2, assign=2)
    s1, s2, s3 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    bd = [dev(b) for b in bs]
    torch.cuda.synchronize()
    outs = []
    for k in range(8):
        st = s1 if k % 2 == 0 else s2
        with torch.cuda.stream(st):
            outs.append(h.solve(bd[k % 4], stream=st))
    v2 = dev(T.vals * 0.5)
    torch.cuda.synchronize()
    with torch.cuda.stream(s3):
        h.update_values(v2, stream=s3)
    with torch.cuda.stream(s1):
        after = h.solve(bd[0], stream=s1)
    torch.cuda.synchronize()
    h.status()
    for k in range(8):
        ref = o.solve(T.row_ptr, T.col_idx, T.vals, bs[k % 4])
        assert relerr(host(outs[k]), ref) <= TOL64, k
    assert relerr(host(after), o.solve(T.row_ptr, T.col_idx, T.vals * 0.5, bs[0])) <= TOL64


@pytest.mark.parametrize("coop", [0, 1])
def test_concurrent_static_grids(sp, coop):
    """Static-schedule solves of four handles issued on four streams with no
    ordering between them, so their persistent grids may share the GPU: each
    grid checks its own residency (its handle's counter), and every result
    equals the same solve run alone, bit for bit."""
    tris = [W.laplacian_triangle((34, 33, 32)), W.laplacian_triangle((34, 33, 32), upper=True),
            W.ilu0_lower((30, 30, 30)), W.powerlaw_lower(30000, 9, window=4000)]
    opts = [dict(algo=2, assign=2, grid=256), dict(algo=2, assign=0, grid=128),
            dict(algo=2, assign=2, grid=512), dict(algo=2, assign=2, grid=512, xp_stride=4)]
    hs = [sp.Handle(*dev_tri(T), uplo="U" if T.upper else "L").configure(cooperative=coop, **o)
          for T, o in zip(tris, opts)]
    bs = [dev(W.uniform_vector(T.n, 70 + k)) for k, T in enumerate(tris)]
    alone = []
    for h, b in zip(hs, bs):
        alone.append(host(h.solve(b)).copy())
        h.status()
    streams = [torch.cuda.Stream() for _ in hs]
    outs = [[torch.empty_like(b) for _ in range(6)] for b in bs]
    torch.cuda.synchronize()
    for r in range(6):
        for h, b, st, o in zip(hs, bs, streams, outs):
            with torch.cuda.stream(st):
                h.solve(b, out=o[r], stream=st)
    torch.cuda.synchronize()
    for k, h in enumerate(hs):
        h.status()
        for r in range(6):
            assert bits_equal(host(outs[k][r]), alone[k]), (k, r)
        h.close()


def test_batched(sp):
    o = oracle.get()
    tris = [W.ilu0_lower((s, s)) for s in (7, 33, 20, 64, 5, 41)]
    tris.append(W.laplacian_triangle((9, 8)))
    bs = [W.uniform_vector(t.n, 40 + i) for i, t in enumerate(tris)]
    devs = [dev_tri(t) for t in tris]
    for opts in (dict(algo=1), dict(algo=2, sync=0), dict(algo=2, sync=1), dict(algo=3)):
        bh = sp.BatchedHandle([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs]).configure(**opts)
        x = host(bh.solve(dev(np.concatenate(bs))))
        bh.status()
        off = 0
        for t, b, d in zip(tris, bs, devs):
            xs = x[off:off + t.n]
            assert relerr(xs, o.solve(t.row_ptr, t.col_idx, t.vals, b)) <= TOL64
            single = sp.Handle(*d).configure(**opts)
            assert bits_equal(xs, host(single.solve(dev(b))))
            off += t.n
    # grad on the concatenated pattern and new values
    new_vals = [d[2] * 0.5 for d in devs]
    bh.update_values(new_vals)
    x = host(bh.solve(dev(np.concatenate(bs))))
    off = 0
    for t, b in zip(tris, bs):
        assert relerr(x[off:off + t.n], o.solve(t.row_ptr, t.col_idx, t.vals * 0.5, b)) <= TOL64
        off += t.n


def test_block_resident_matches_streamed(sp):
    """Whole systems in LDS (the 2-D 64x64 triangle; a batch of small ILU(0)
    and mesh factors) against the streamed block kernel bit for bit, both
    directions, and against the oracle."""
    o = oracle.get()
    for tris in ([W.c1_lap2d_64()[0]],
                 [W.ilu0_lower((9, 14)), W.laplacian_triangle((5, 4, 3)), W.ilu0_lower((30, 31)),
                  W.ilu0_lower((1, 1))]):
        devs = [dev_tri(t) for t in tris]
        bs = [W.uniform_vector(t.n, 80 + i) for i, t in enumerate(tris)]
        bb = dev(np.concatenate(bs))
        mk = lambda **kw: sp.BatchedHandle([d[0] for d in devs], [d[1] for d in devs],
                                           [d[2] for d in devs]).configure(algo=3, **kw)
        hr, hs = mk(), mk(block_resident=0)
        assert hr.get_option("block_resident") == 1 and hs.get_option("block_resident") == 0
        x, xt = hr.solve(bb), hr.solve_t(bb)
        assert bits_equal(x, hs.solve(bb)) and bits_equal(xt, hs.solve_t(bb))
        x, xt = host(x), host(xt)
        off = 0
        for t, b in zip(tris, bs):
            assert relerr(x[off:off + t.n], o.solve(t.row_ptr, t.col_idx, t.vals, b)) <= TOL64
            assert relerr(xt[off:off + t.n],
                          o.solve_transpose(t.row_ptr, t.col_idx, t.vals, b)) <= TOL64
            off += t.n
        hr.status()
        hs.status()


def test_block_resident_signed_zeros(sp):
    """Products that underflow to zeros of either sign and b entries of -0:
    the resident kernel's dummy entries (value -0) must leave every sum's
    bits alone, so both block kernels agree bit for bit, zero signs included."""
    T = W.c1_lap2d_64()[0]
    rows = np.repeat(np.arange(T.n), np.diff(T.row_ptr))
    v = np.where(T.col_idx == rows, 1.0, T.vals * 1e-200)
    b = W.uniform_vector(T.n, 31) * 1e-200
    b[::10] = -0.0
    xs = []
    for r in (1, 0):
        h = sp.Handle(dev(T.row_ptr), dev(T.col_idx), dev(v)).configure(algo=3, block_resident=r)
        xs.append(h.solve(dev(b)))
        h.status()
    assert bits_equal(xs[0], xs[1])
    xh = host(xs[0])
    assert np.signbit(xh).any() and (xh == 0).any()     # the case is exercised


def test_default_schedule_follows_the_pattern(sp):
    """Without tuning or schedule options the schedule follows features of
    the pattern, and every such choice gives the bits of an explicitly chosen
    one-lane-per-row (or same lane rule) schedule."""
    o = oracle.get()
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    cases = [(W.c1_lap2d_64()[0], dict(algo=3)),                            # whole system in LDS
             (W.powerlaw_lower(50000, 21, window=5000),
              dict(algo=2, grid=2 * cu, xp_stride=4, assign=2)),             # long rows
             (W.laplacian_triangle((30, 30, 30)), dict(algo=2, assign=1))]   # narrow levels
    for T, want in cases:
        b = W.uniform_vector(T.n, 17)
        h = sp.Handle(*dev_tri(T))
        info = h.info()
        for k, v in want.items():
            assert info[k] == v, (T.name, k, info[k], v)
        x = h.solve(dev(b))
        h.status()
        ref = sp.Handle(*dev_tri(T)).configure(algo=2, assign=0, grid=0, xp_stride=1)
        assert bits_equal(x, ref.solve(dev(b)))
        assert relerr(host(x), o.solve(T.row_ptr, T.col_idx, T.vals, b)) <= TOL64
        # an option set explicitly is kept
        assert h.configure(assign=0).info()["assign"] == 0


def test_block_global_x_path(sp):
    """A batch whose largest system does not fit in LDS (x in global memory),
    against the oracle and bitwise against the one-lane-per-row level solve."""
    o = oracle.get()
    tris = [W.ilu0_lower((150, 150)), W.ilu0_lower((40, 37)), W.laplacian_triangle((9, 8, 7))]
    bs = [W.uniform_vector(t.n, 60 + i) for i, t in enumerate(tris)]
    devs = [dev_tri(t) for t in tris]
    bb = dev(np.concatenate(bs))
    hb = sp.BatchedHandle([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs]).configure(algo=3)
    hl = sp.BatchedHandle([d[0] for d in devs], [d[1] for d in devs], [d[2] for d in devs]).configure(algo=1, group=1)
    x = hb.solve(bb)
    assert bits_equal(x, hl.solve(bb))
    xt = host(hb.solve_t(bb))
    x = host(x)
    off = 0
    for t, b in zip(tris, bs):
        assert relerr(x[off:off + t.n], o.solve(t.row_ptr, t.col_idx, t.vals, b)) <= TOL64
        assert relerr(xt[off:off + t.n], o.solve_transpose(t.row_ptr, t.col_idx, t.vals, b)) <= TOL64
        off += t.n
    hb.status()


def test_update_values_and_zero_pivot(sp):
    o = oracle.get()
    T = W.laplacian_triangle((10, 9, 8))
    rp, ci, v = dev_tri(T)
    h = sp.Handle(rp, ci, v)
    h.prepare_transpose()
    hb = sp.Handle(rp, ci, v).configure(algo=3)
    hb.solve_t(dev(np.ones(T.n)))         # builds both block plans before the update
    hb.solve(dev(np.ones(T.n)))
    v2 = T.vals * np.linspace(0.5, 2.0, T.nnz)
    h.update_values(dev(v2))
    hb.update_values(dev(v2))
    b = W.uniform_vector(T.n, 1)
    for hh in (h, hb):
        assert relerr(host(hh.solve(dev(b))), o.solve(T.row_ptr, T.col_idx, v2, b)) <= TOL64
        assert relerr(host(hh.solve_t(dev(b))), o.solve_transpose(T.row_ptr, T.col_idx, v2, b)) <= TOL64
    vz = v2.copy()
    vz[T.row_ptr[5 + 1] - 1] = 0.0          # diagonal of row 5 (stored last)
    h.update_values(dev(vz))
    with pytest.raises(sp.SpTRSVError) as e:
        h.status()
    assert e.value.status == -7
    with pytest.raises(sp.SpTRSVError) as e:
        sp.Handle(rp, ci, dev(vz))
    assert e.value.status == -7


def test_validation_errors(sp):
    T = W.laplacian_triangle((4, 4))
    rp, ci, v = T.row_ptr, T.col_idx, T.vals
    with pytest.raises(sp.SpTRSVError) as e:
        sp.Handle(dev(rp), dev(ci), dev(v), uplo="U")
    assert e.value.status == -4
    bad = ci.copy(); bad[3] = 99
    with pytest.raises(sp.SpTRSVError) as e:
        sp.Handle(dev(rp), dev(bad), dev(v))
    assert e.value.status == -3
    rp2 = rp.copy(); rp2[1:] -= 1
    with pytest.raises(sp.SpTRSVError) as e:
        sp.Handle(dev(rp2), dev(ci[1:]), dev(v[1:]))
    assert e.value.status == -6


def test_binding_rejects_short_buffers(sp):
    """Buffers of the wrong length or type are refused before any launch (a
    kernel would otherwise read or write past their end)."""
    T = W.laplacian_triangle((6, 5))
    n = T.n
    with pytest.raises(ValueError):
        sp.Handle(dev(T.row_ptr), dev(T.col_idx), dev(T.vals[:-1]))
    h = sp.Handle(dev(T.row_ptr), dev(T.col_idx), dev(T.vals))
    b = dev(np.ones(n))
    for bad in (torch.empty(n - 1, dtype=torch.float64, device=DEV),
                torch.empty(n, dtype=torch.float32, device=DEV)):
        with pytest.raises((ValueError, TypeError)):
            h.solve(b, out=bad)
        with pytest.raises((ValueError, TypeError)):
            h.solve_t(bad)
        with pytest.raises((ValueError, TypeError)):
            h.tune(b, bad)
        with pytest.raises((ValueError, TypeError)):
            h.capture(b, bad)
        with pytest.raises((ValueError, TypeError)):
            h.grad_vals(b, bad)
    with pytest.raises(ValueError):
        h.update_values(dev(T.vals[:-2]))
    for bad_stride in (0, 3, 32):
        with pytest.raises(sp.SpTRSVError):
            h.set_option("xp_stride", bad_stride)
    with pytest.raises(ValueError):
        h.grad_vals(b, b, out=torch.empty(T.nnz - 1, dtype=torch.float64, device=DEV))
    bh = sp.BatchedHandle([dev(T.row_ptr)] * 2, [dev(T.col_idx)] * 2, [dev(T.vals)] * 2)
    with pytest.raises(ValueError):
        bh.update_values([dev(T.vals)])
    with pytest.raises(ValueError):
        bh.update_values([dev(T.vals), dev(T.vals[:-1])])
    # the handle still solves correctly after the refused calls
    x = host(h.solve(b))
    ref = oracle.get().solve(T.row_ptr, T.col_idx, T.vals, np.ones(n))
    assert relerr(x, ref) <= TOL64


def test_empty_and_single(sp):
    h = sp.Handle(dev(np.zeros(1, np.int32)), dev(np.zeros(0, np.int32)), dev(np.zeros(0)))
    x = h.solve(dev(np.zeros(0)))
    assert x.numel() == 0
    h.status()
    h = sp.Handle(dev(np.array([0, 1], np.int32)), dev(np.array([0], np.int32)), dev(np.array([4.0])))
    for algo in (1, 2):
        h.set_option("algo", algo)
        assert host(h.solve(dev(np.array([2.0]))))[0] == 0.5


@pytest.mark.parametrize("sync,assign,poll", [(0, 0, 1), (0, 0, 0), (0, 1, 1), (1, 1, 1)])
def test_watchdog_timeout_is_reported_and_recovers(sp, sync, assign, poll):
    """A spin limit of one poll (forced from the host) makes waits give up:
    the kernel drains, TIMEOUT is reported; with the default limit the same
    handle solves correctly again."""
    n = 20000
    P = W.bidiagonal_fast(n, 1.0, 1.0)
    b = np.ones(n)
    h = sp.Handle(*dev_tri(P)).configure(algo=2, sync=sync, assign=assign, spin_limit=1, poll=poll)
    h.solve(dev(b))
    with pytest.raises(sp.SpTRSVError) as e:
        h.status()
    assert e.value.status == -10
    h.set_option("spin_limit", 1 << 22)
    x = host(h.solve(dev(b)))
    h.status()
    assert np.array_equal(x, np.arange(1, n + 1, dtype=np.float64))


@pytest.mark.parametrize("coop", [0, 1])
@pytest.mark.parametrize("opts,nrhs", [(dict(algo=2, assign=0, grid=16), 1),
                                       (dict(algo=2, assign=2, grid=64), 1),
                                       (dict(algo=2, assign=0, grid=32, wg=256), 1),
                                       (dict(algo=2, assign=0, grid=24), 16),
                                       (dict(algo=5, assign=0, grid=16), 1)])
def test_residency_check_forced(sp, opts, nrhs, coop):
    """The static schedules' residency check, forced to fail from the host
    (limit 0: every wavefront but the last to sign in gives up), with an
    ordinary and with a cooperative launch: the grid drains, the status is
    NOT_RESIDENT (distinct from the wait watchdog's TIMEOUT), and with the
    default limit the same handle solves correctly again."""
    T = W.laplacian_triangle((30, 28, 26))
    o = oracle.get()
    F = np.stack([W.uniform_vector(T.n, 60 + r) for r in range(nrhs)], 0)
    h = sp.Handle(*dev_tri(T)).configure(residency_limit=0, cooperative=coop, **opts)
    run = (lambda: h.solve(dev(F[0]))) if nrhs == 1 else (lambda: h.solve_multi(dev(F)))
    run()
    with pytest.raises(sp.SpTRSVError) as e:
        h.status()
    assert e.value.status == -14
    h.set_option("residency_limit", 1 << 20)
    X = host(run()).reshape(nrhs, T.n)
    h.status()
    Xo = o.solve_multi(T.row_ptr, T.col_idx, T.vals, F.T)
    assert relerr(X.T, Xo) <= TOL64


@pytest.mark.parametrize("opts,nrhs", [(dict(algo=2, assign=0, grid=64), 1),
                                       (dict(algo=2, assign=2, grid=256), 1),
                                       (dict(algo=2, assign=2, grid=128, xp_stride=4), 1),
                                       (dict(algo=2, assign=0, grid=96), 16)])
def test_cooperative_launch_same_bits(sp, opts, nrhs):
    """The persistent static grids launched cooperatively and ordinarily
    (the default) give the same bits, forward and transposed, and match the
    oracle; the option reads back."""
    T = W.laplacian_triangle((31, 29, 27))
    o = oracle.get()
    F = np.stack([W.uniform_vector(T.n, 80 + r) for r in range(nrhs)], 0)
    out = {}
    for coop in (0, 1):
        h = sp.Handle(*dev_tri(T)).configure(cooperative=coop, **opts)
        assert h.get_option("cooperative") == coop
        with pytest.raises(sp.SpTRSVError):
            h.set_option("cooperative", 2)
        assert h.get_option("cooperative") == coop
        if nrhs == 1:
            fwd, trn = h.solve(dev(F[0])), h.solve_t(dev(F[0]))
        else:
            fwd, trn = h.solve_multi(dev(F)), h.solve_multi(dev(F), transpose=True)
        h.status()
        out[coop] = (host(fwd).copy(), host(trn).copy())
        h.close()
    for k in range(2):
        assert np.array_equal(out[0][k].view(np.uint8), out[1][k].view(np.uint8)), k
    Xo = o.solve_multi(T.row_ptr, T.col_idx, T.vals, F.T)
    assert relerr(out[0][0].reshape(nrhs, T.n).T, Xo) <= TOL64


def test_column_self_cooperative_launch(sp):
    """The column-wise self-scheduled solve (one persistent grid) in both
    launch modes: same result as the oracle to rounding (its update order
    follows timing, so not bit for bit)."""
    T = W.laplacian_triangle((30, 28, 26))
    o = oracle.get()
    b = W.uniform_vector(T.n, 91)
    xo = o.solve(T.row_ptr, T.col_idx, T.vals, b, False)
    for coop in (0, 1):
        h = sp.Handle(*dev_tri(T)).configure(algo=5, cooperative=coop)
        x = host(h.solve(dev(b)))
        h.status()
        assert relerr(x, xo) <= TOL64, coop
        h.close()


@pytest.mark.parametrize("opts", [dict(algo=1), dict(algo=2, sync=0), dict(algo=2, sync=1),
                                  dict(algo=3),
                                  dict(algo=2, sync=0, xp_stride=2),
                                  dict(algo=2, sync=0, assign=2, cooperative=1)])
def test_graph_replay(sp, opts):
    T = W.laplacian_triangle((24, 23, 22))
    h = sp.Handle(*dev_tri(T)).configure(**opts)
    s = torch.cuda.Stream()
    b = dev(W.uniform_vector(T.n, 2))
    x = torch.empty_like(b)
    with torch.cuda.stream(s):
        ref = h.solve(b)
        g = h.capture(b, x, stream=s)
        gt = h.capture(b, x, transpose=True, stream=s)
        ref_t = h.solve_t(b)
        for rep in range(5):
            x.zero_()
            g.launch(s)
            s.synchronize()
            assert bits_equal(x, ref), rep
            junk = h.solve(b * 2.0)            # eager work between replays
            s.synchronize()
            gt.launch(s)
            s.synchronize()
            assert bits_equal(x, ref_t), rep
    h.status()


@pytest.mark.parametrize("case", ["block_in_lds", "long_rows_static", "narrow_ticket"])
def test_graph_replay_default_schedules(sp, case):
    """Graphs of the schedules the pattern picks by default (the whole
    system in LDS; the XCD-regional static schedule with 32-byte slots; the
    ticket schedule), captured before any eager solve, replayed with eager
    work in between, against the eager solve bit for bit."""
    T = {"block_in_lds": W.c1_lap2d_64()[0],
         "long_rows_static": W.powerlaw_lower(30000, 19, window=3000),
         "narrow_ticket": W.laplacian_triangle((24, 23, 22))}[case]
    h = sp.Handle(*dev_tri(T))
    want = {"block_in_lds": dict(algo=3), "long_rows_static": dict(algo=2, assign=2, xp_stride=4),
            "narrow_ticket": dict(algo=2, assign=1)}[case]
    info = h.info()
    assert all(info[k] == v for k, v in want.items()), info
    s = torch.cuda.Stream()
    b = dev(W.uniform_vector(T.n, 5))
    x = torch.empty_like(b)
    with torch.cuda.stream(s):
        g = h.capture(b, x, stream=s)
        ref = h.solve(b)
        for rep in range(4):
            x.zero_()
            g.launch(s)
            s.synchronize()
            assert bits_equal(x, ref), rep
            h.solve(b * 3.0)                   # eager work between replays
            s.synchronize()
    h.status()


def test_capture_first_with_xp_stride(sp):
    """A graph captured before any eager solve, with values in 8-byte slots:
    the wider solution buffer is sized before the capture."""
    T = W.laplacian_triangle((19, 18, 17))
    v32 = T.vals.astype(np.float32)
    h = sp.Handle(dev(T.row_ptr), dev(T.col_idx), dev(v32)).configure(algo=2, sync=0,
                                                                        xp_stride=2)
    assert h.info()["xp_stride"] == 2
    s = torch.cuda.Stream()
    b = dev(W.uniform_vector(T.n, 4).astype(np.float32))
    x = torch.empty_like(b)
    with torch.cuda.stream(s):
        g = h.capture(b, x, stream=s)
        for rep in range(3):
            x.zero_()
            g.launch(s)
            s.synchronize()
            ref = h.solve(b)
            s.synchronize()
            assert bits_equal(x, ref), rep
    h.status()
    xo = oracle.get().solve(T.row_ptr, T.col_idx, v32.astype(np.float64),
                            host(b).astype(np.float64))
    assert relerr(host(x), xo) <= TOL32


def test_tune_and_timing(sp):
    o = oracle.get()
    T = W.laplacian_triangle((30, 30, 30))
    h = sp.Handle(*dev_tri(T))
    b = dev(W.uniform_vector(T.n, 3))
    info = h.tune(b)
    assert info["algo"] in (1, 2)
    h.set_option("timing", 1)
    for _ in range(4):
        x = h.solve(b)
    ms, cnt = h.kernel_time()
    assert cnt == 4 and ms > 0
    assert relerr(host(x), o.solve(T.row_ptr, T.col_idx, T.vals, host(b))) <= TOL64


def test_probe_hop(sp):
    """The hop probe returns a plausible latency for both placements."""
    for same in (True, False):
        ns = sp.probe_hop(same_xcd=same, iters=200)
        assert 10.0 < ns < 1e5, (same, ns)


def test_mixed_solve_sequence(sp):
    """A mixed sequence on one handle (slot widths of the position-ordered
    solution, several right-hand sides, level scheduling, tickets,
    transposes) gives every solve bit for bit what a fresh handle gives: no
    state left by one solve leaks into the next."""
    T = W.laplacian_triangle((21, 17, 13))
    b = dev(W.uniform_vector(T.n, 12))
    F = dev(np.stack([W.uniform_vector(T.n, 20 + r) for r in range(3)]))

    def fresh(**opts):
        return sp.Handle(*dev_tri(T)).configure(**opts)

    want = {}
    for key, opts in (("s1", dict(algo=2, sync=0, assign=0)),
                      ("s4", dict(algo=2, sync=0, assign=2, xp_stride=4)),
                      ("lv", dict(algo=1)),
                      ("tk", dict(algo=2, sync=0, assign=1))):
        want[key] = fresh(**opts).solve(b)
        want[key + "t"] = fresh(**opts).solve_t(b)
    want["multi"] = fresh(algo=2, sync=0, assign=0).solve_multi(F)
    h = sp.Handle(*dev_tri(T))
    seq = ["s1", "s1", "s4", "lv", "s1", "multi", "s4", "tk", "s1t", "s4t", "multi", "lvt",
           "s1", "tkt", "s4"]
    opts_of = {"s1": dict(algo=2, sync=0, assign=0, xp_stride=1),
               "s4": dict(algo=2, sync=0, assign=2, xp_stride=4),
               "lv": dict(algo=1), "tk": dict(algo=2, sync=0, assign=1, xp_stride=1)}
    for it, key in enumerate(seq):
        if key == "multi":
            h.configure(algo=2, sync=0, assign=0, xp_stride=1)
            assert bits_equal(h.solve_multi(F), want["multi"]), it
            continue
        base = key.rstrip("t")
        h.configure(**opts_of[base])
        got = h.solve_t(b) if key.endswith("t") else h.solve(b)
        assert bits_equal(got, want[key]), (it, key)
    h.status()
