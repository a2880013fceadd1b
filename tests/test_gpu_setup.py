"""Device setup route (levels, level sets, level-ordered layout computed on
the GPU) against the CPU oracle and against the host route.

Bars: exported analysis (levels, ilev, jlev, depcnt) bit-exact against the
oracle, for T and for T^T; solves bitwise equal to the host route's (both
routes produce the same plan, so every schedule runs the same arithmetic);
invalid and unsorted patterns handed to the host route with its error.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpuhelp import bits_equal, dev, dev_tri, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_1710_04985_amd as sp
    assert torch.cuda.is_available()
    return sp


def _drop_diagonal(T):
    """T without its stored diagonal (for unit_diag with no diagonal stored)."""
    rows = np.repeat(np.arange(T.n), np.diff(T.row_ptr))
    keep = T.col_idx != rows
    rp = np.zeros(T.n + 1, np.int32)
    rp[1:] = np.cumsum(np.bincount(rows[keep], minlength=T.n))
    return W.Triangle(T.n, rp, T.col_idx[keep].astype(np.int32), T.vals[keep], upper=T.upper,
                      unit_diag=True, name=T.name + "_nodiag")


CASES = [("c1_lap2d_64", W.c1_lap2d_64()[0]),
         ("lap3d_20_L", W.laplacian_triangle((20, 20, 20))),
         ("lap3d_17x9x5_U", W.laplacian_triangle((17, 9, 5), upper=True)),
         ("powerlaw_50k", W.powerlaw_lower(50000, 21, window=5000)),
         ("ilu0_12", W.ilu0_lower((12, 12, 12))),
         ("st9_30x20_L", W.stencil_triangle((30, 20), 9)),
         ("st27_12x11x10_U", W.stencil_triangle((12, 11, 10), 27, upper=True)),
         ("dense_rand_300_U", W.random_triangle(300, 7, density=0.6, upper=True)),
         ("dense_rand_200_L", W.random_triangle(200, 8, density=0.9)),
         ("chain_5000", W.bidiagonal_fast(5000, 2.0, 1.0)),
         ("chain_5000_U", W.bidiagonal_fast(5000, 2.0, 1.0, upper=True)),
         ("diag_1000", W.diagonal_matrix(np.linspace(1.0, 2.0, 1000))),
         ("single", W.diagonal_matrix([3.0])),
         ("unit_nodiag", _drop_diagonal(W.laplacian_triangle((9, 8, 7))))]


def _handle(sp, T, setup, dtype=torch.float64):
    return sp.Handle(*dev_tri(T, dtype), uplo="U" if T.upper else "L", unit_diag=T.unit_diag,
                     setup=setup)


@pytest.mark.parametrize("name,T", CASES, ids=[c[0] for c in CASES])
def test_device_analysis_bit_exact(sp, name, T):
    print("device setup", name, T.n, flush=True)
    o = oracle.get()
    h = _handle(sp, T, "device")
    route, ms = h.setup_info()
    assert route == "device" and ms >= 0.0
    lv, nlev, il, jl, dc = o.analyze(T.row_ptr, T.col_idx, T.upper)
    assert h.info()["nlev"] == nlev
    level, ilev, jlev, dep = h.export_analysis()
    assert np.array_equal(level, lv) and np.array_equal(ilev, il)
    assert np.array_equal(jlev, jl) and np.array_equal(dep, dc)
    rT, cT, _ = o.transpose(T.row_ptr, T.col_idx)
    lvT, nlevT, ilT, jlT, dcT = o.analyze(rT, cT, not T.upper)
    level, ilev, jlev, dep = h.export_analysis(transpose=True)
    assert np.array_equal(level, lvT) and np.array_equal(ilev, ilT)
    assert np.array_equal(jlev, jlT) and np.array_equal(dep, dcT)


SCHEDULES = [dict(algo=1), dict(algo=2), dict(algo=2, assign=1), dict(algo=2, assign=2),
             dict(algo=3)]


@pytest.mark.parametrize("name,T", CASES, ids=[c[0] for c in CASES])
def test_device_route_solves_match_host_route(sp, name, T):
    print("device vs host route", name, T.n, flush=True)
    hd = _handle(sp, T, "device")
    hh = _handle(sp, T, "host")
    assert hh.setup_info()[0] == "host"
    rng = np.random.default_rng(3)
    b = dev(rng.uniform(-1, 1, T.n))
    for opts in SCHEDULES:
        for k, v in opts.items():
            hd.set_option(k, v)
            hh.set_option(k, v)
        assert bits_equal(hd.solve(b), hh.solve(b)), opts
        assert bits_equal(hd.solve_t(b), hh.solve_t(b)), opts
    hd.status()
    hh.status()
    # the solution itself against the oracle
    x = host(hd.solve(b))
    ref = oracle.get().solve(T.row_ptr, T.col_idx, T.vals, host(b), T.upper, T.unit_diag)
    assert np.abs(x - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300)


def test_device_route_fp32_and_multi(sp):
    T = W.laplacian_triangle((16, 15, 14), upper=True)
    for dt in (torch.float64, torch.float32):
        hd = _handle(sp, T, "device", dt)
        hh = _handle(sp, T, "host", dt)
        B = dev(np.random.default_rng(4).uniform(-1, 1, (5, T.n)), dt)
        assert bits_equal(hd.solve(B[0]), hh.solve(B[0]))
        assert bits_equal(hd.solve_multi(B), hh.solve_multi(B))
        assert bits_equal(hd.solve_multi(B, transpose=True), hh.solve_multi(B, transpose=True))


def test_unsorted_rows_take_the_host_route(sp):
    T = W.random_triangle(300, 5, density=0.05, upper=True, shuffle_rows=True)
    h = _handle(sp, T, "device")
    assert h.setup_info()[0] == "host"
    level, ilev, jlev, dep = h.export_analysis()
    lv, nlev, il, jl, dc = oracle.get().analyze(T.row_ptr, T.col_idx, T.upper)
    assert np.array_equal(level, lv) and np.array_equal(jlev, jl)


def _status(sp, rp, ci, v, uplo, setup):
    try:
        sp.Handle(dev(rp), dev(ci), dev(v), uplo=uplo, setup=setup)
    except sp.SpTRSVError as e:
        return e.status
    return 0


def test_invalid_patterns_report_the_host_error(sp):
    T = W.laplacian_triangle((4, 4))
    rp, ci, v = T.row_ptr, T.col_idx, T.vals
    bad = ci.copy(); bad[3] = 99
    rp2 = rp.copy(); rp2[1:] -= 1
    dup = ci.copy(); dup[4] = dup[3]
    swap = ci.copy(); swap[[3, 4]] = swap[[4, 3]]
    vz = v.copy(); vz[rp[3] - 1] = 0.0
    rpx = rp.copy(); rpx[2] = rpx[3] + 1
    cases = [(rp, ci, v, "U", -4), (rp, bad, v, "L", -3), (rp2, ci[1:], v[1:], "L", -6),
             (rp, dup, v, "L", None), (rp, swap, v, "L", 0), (rp, ci, vz, "L", -7),
             (rpx, ci, v, "L", -2)]
    for k, (r, c, vv, uplo, want) in enumerate(cases):
        sd = _status(sp, r, c, vv, uplo, "device")
        sh = _status(sp, r, c, vv, uplo, "host")
        assert sd == sh, (k, sd, sh)
        if want is not None:
            assert sd == want, (k, sd)
        else:
            assert sd < 0


@pytest.mark.parametrize("upper", [False, True], ids=["L", "U"])
def test_device_analysis_full_size_lap3d128(sp, upper):
    """The 128^3 7-point triangles (2,097,152 rows, 382 levels)."""
    print("device setup lap3d 128", "U" if upper else "L", flush=True)
    T = W.laplacian_triangle((128, 128, 128), upper=upper)
    h = _handle(sp, T, "device")
    assert h.setup_info()[0] == "device"
    lv, nlev, il, jl, dc = oracle.get().analyze(T.row_ptr, T.col_idx, T.upper)
    assert nlev == 382 and h.info()["nlev"] == 382
    level, ilev, jlev, dep = h.export_analysis()
    assert np.array_equal(level, lv) and np.array_equal(ilev, il)
    assert np.array_equal(jlev, jl) and np.array_equal(dep, dc)


def test_device_analysis_full_size_powerlaw(sp):
    """The random power-law triangle (10^6 rows, rows of up to ~2000
    dependencies): its long rows take the level sweep's whole-wavefront
    reads.  Levels, level sets and counts bit-exact; the solve matches the
    host route's bit for bit."""
    print("device setup power-law 1e6", flush=True)
    T, xs, b = W.c3_powerlaw()
    h = _handle(sp, T, "device")
    assert h.setup_info()[0] == "device"
    lv, nlev, il, jl, dc = oracle.get().analyze(T.row_ptr, T.col_idx, T.upper)
    assert h.info()["nlev"] == nlev
    level, ilev, jlev, dep = h.export_analysis()
    assert np.array_equal(level, lv) and np.array_equal(ilev, il)
    assert np.array_equal(jlev, jl) and np.array_equal(dep, dc)
    hh = _handle(sp, T, "host")
    assert bits_equal(h.solve(dev(b)), hh.solve(dev(b)))


def _batch(seed, count, lo, hi):
    rng = np.random.default_rng(seed)
    tris = []
    for k in range(count):
        sx, sy = (int(v) for v in rng.integers(lo, hi + 1, 2))
        T = W.ilu0_lower((sx, sy))
        T.vals = T.vals * W.uniform_vector(T.nnz, 100 + k, 0.9, 1.1)
        tris.append(T)
    return tris


def _batched(sp, tris, setup, **kw):
    d = [dev_tri(t) for t in tris]
    return sp.BatchedHandle([x[0] for x in d], [x[1] for x in d], [x[2] for x in d], setup=setup,
                            **kw)


def test_batched_device_route(sp):
    """The batch concatenated and analysed in device memory: analysis of the
    concatenation (and of its transpose) bit-exact against the oracle, every
    schedule's solve, transposed solve and value gradient bitwise equal to the
    host route's."""
    o = oracle.get()
    tris = _batch(5, 24, 4, 40)
    hd = _batched(sp, tris, "device")
    hh = _batched(sp, tris, "host")
    assert hd.setup_info()[0] == "device" and hh.setup_info()[0] == "host"
    C = W.concat_block_diagonal(tris)
    lv, nlev, il, jl, dc = o.analyze(C.row_ptr, C.col_idx, False)
    level, ilev, jlev, dep = hd.export_analysis()
    assert np.array_equal(level, lv) and np.array_equal(ilev, il)
    assert np.array_equal(jlev, jl) and np.array_equal(dep, dc)
    rT, cT, _ = o.transpose(C.row_ptr, C.col_idx)
    lvT, _, ilT, jlT, dcT = o.analyze(rT, cT, True)
    level, ilev, jlev, dep = hd.export_analysis(transpose=True)
    assert np.array_equal(level, lvT) and np.array_equal(ilev, ilT)
    assert np.array_equal(jlev, jlT) and np.array_equal(dep, dcT)
    b = dev(W.uniform_vector(C.n, 6))
    for opts in SCHEDULES:
        hd.configure(**opts)
        hh.configure(**opts)
        assert bits_equal(hd.solve(b), hh.solve(b)), opts
        assert bits_equal(hd.solve_t(b), hh.solve_t(b)), opts
    x = hd.solve(b)
    gb = hd.solve_t(b)
    assert bits_equal(hd.grad_vals(gb, x), hh.grad_vals(gb, x))
    hd.status()
    hh.status()
    assert np.abs(host(x) - o.solve(C.row_ptr, C.col_idx, C.vals, host(b))).max() <= \
        1e-12 * np.abs(host(x)).max()


def test_batched_device_route_invalid_system(sp):
    """A system whose column lies outside it (but inside the concatenation)
    and one with a bad row pointer: the device route hands them to the host
    route, which reports the same error either way."""
    tris = _batch(7, 5, 3, 6)
    for k, mutate, want in ((2, "col", -4), (3, "rp", -2)):
        bad = [W.Triangle(t.n, t.row_ptr.copy(), t.col_idx.copy(), t.vals.copy()) for t in tris]
        if mutate == "col":
            bad[k].col_idx[bad[k].row_ptr[1]] = bad[k].n + 1   # past its own system
        else:
            bad[k].row_ptr[-1] -= 1
        got = []
        for setup in ("device", "host"):
            try:
                _batched(sp, bad, setup)
                got.append(0)
            except sp.SpTRSVError as e:
                got.append(e.status)
        assert got[0] == got[1] and got[0] < 0, (mutate, got)


def test_batched_device_route_full_size_c4a(sp):
    """The 256 ILU(0) factors at full size on the device route: analysis
    bit-exact against the host route's plan (solves bitwise equal)."""
    print("batched device setup C4a", flush=True)
    tris, xs, bs = W.c4a_batch()
    hd = _batched(sp, tris, "device")
    route, ms = hd.setup_info()
    print("C4a device setup %.1f ms" % ms, flush=True)
    assert route == "device"
    hh = _batched(sp, tris, "host")
    b = dev(np.concatenate(bs))
    for opts in (dict(algo=2), dict(algo=1)):
        hd.configure(**opts)
        hh.configure(**opts)
        assert bits_equal(hd.solve(b), hh.solve(b))
    hd.status()


def test_transpose_on_device_full_size_ilu96(sp):
    """The 96^3 ILU(0) factor analysed on the device: its transposed
    analysis (the adjoint's) is also built on the device, bit-exact against
    the oracle's analysis of T^T, and the transposed solve equals the host
    route's bit for bit."""
    print("device transpose ILU(0) 96^3", flush=True)
    o = oracle.get()
    T = W.c5_ilu3d()[0]
    h = _handle(sp, T, "device")
    h.prepare_transpose()
    rT, cT, _ = o.transpose(T.row_ptr, T.col_idx)
    lvT, nlevT, ilT, jlT, dcT = o.analyze(rT, cT, True)
    level, ilev, jlev, dep = h.export_analysis(transpose=True)
    assert nlevT == 286
    assert np.array_equal(level, lvT) and np.array_equal(ilev, ilT)
    assert np.array_equal(jlev, jlT) and np.array_equal(dep, dcT)
    g = dev(W.uniform_vector(T.n, 9))
    hh = _handle(sp, T, "host")
    assert bits_equal(h.solve_t(g), hh.solve_t(g))
    h.status()
