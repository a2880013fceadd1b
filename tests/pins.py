"""Pins of the CPU oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code.

Each pin takes an ``oracle.Oracle`` and raises AssertionError on a mismatch.
They are collected twice: once against the real oracle (test_oracle_pins.py)
and once against copies of the oracle with planted mistakes
(test_oracle_mutants.py), where at least one pin must fail per mistake.
Sizes are tiny so the whole set runs in a few seconds.
"""
from __future__ import annotations

import itertools
import os

import numpy as np
import scipy.linalg as sla

import workloads as W

U64 = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _grid_level(dims, upper):
    """Closed form of the level of node (ix, iy[, iz]) of a 5/7-point
    Laplacian triangle: every stencil edge raises the level by exactly one,
    so the level is the Manhattan distance to the first (lower) or last
    (upper) grid corner.  Summed, it gives Sec. 4.1's nlev formulas."""
    idx = np.arange(int(np.prod(dims)))
    lev = np.zeros_like(idx)
    rem = idx
    for d in dims:
        c = rem % d
        rem = rem // d
        lev = lev + ((d - 1 - c) if upper else c)
    return lev


GRIDS_2D = [(5, 5), (7, 3), (1, 6), (8, 1), (4, 9)]
GRIDS_3D = [(4, 3, 5), (2, 2, 2), (1, 1, 7), (3, 1, 4), (5, 5, 5)]


def pin_levels_closed_form(o):
    """Sec. 4.1: nlev = nx+ny-1 (2-D 5-pt), nx+ny+nz-2 (3-D 7-pt), and the
    per-node distance form; both level formulas, lower and upper."""
    for dims in GRIDS_2D + GRIDS_3D:
        expect_nlev = sum(dims) - (1 if len(dims) == 2 else 2)
        for upper in (False, True):
            T = W.laplacian_triangle(dims, upper=upper)
            for fn in (o.levels_row, o.levels_col):
                level, nlev = fn(T.row_ptr, T.col_idx, upper)
                assert nlev == expect_nlev, (dims, upper, fn.__name__, nlev)
                assert np.array_equal(level, _grid_level(dims, upper)), (dims, upper, fn.__name__)


def _stencil_level(dims, upper):
    """Closed form for the 9-point (2-D) and 27-point (3-D) triangles with
    lexicographic numbering, derived from the longest stencil chains: the
    diagonal neighbour (x+1, y-1) forces two levels per y step when nx >= 2,
    and (x+1, y+1, z-1) forces a + 2 per z step, so
    level = x + a*y (+ b*z), a = 1 + [nx>=2], b = 1 + [nx>=2] + a*[ny>=2];
    mirrored (n_d - 1 - coordinate) for the upper triangle."""
    n = int(np.prod(dims))
    idx = np.arange(n)
    c, rem = [], idx
    for d in dims:
        cc = rem % d
        c.append((d - 1 - cc) if upper else cc)
        rem = rem // d
    a = 1 + (dims[0] >= 2)
    lev = c[0] + a * c[1]
    if len(dims) == 3:
        b = 1 + (dims[0] >= 2) + a * (dims[1] >= 2)
        lev = lev + b * c[2]
    return lev


def pin_levels_stencil9_27(o):
    """Levels of the 9-point and 27-point triangles (Sec. 5.1 stencils)."""
    for dims in [(5, 4), (1, 6), (7, 1), (2, 2), (6, 3)]:
        for upper in (False, True):
            T = W.stencil_triangle(dims, 9, upper=upper)
            level, nlev = o.levels_row(T.row_ptr, T.col_idx, upper)
            want = _stencil_level(dims, upper)
            assert np.array_equal(level, want), (dims, upper)
            assert nlev == int(want.max()) + 1
    for dims in [(4, 3, 5), (3, 1, 4), (1, 3, 3), (1, 1, 5), (2, 2, 2), (5, 4, 3)]:
        for upper in (False, True):
            T = W.stencil_triangle(dims, 27, upper=upper)
            level, nlev = o.levels_row(T.row_ptr, T.col_idx, upper)
            assert np.array_equal(level, _stencil_level(dims, upper)), (dims, upper)


def _read_golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split(":", 1)
            out[k.strip()] = [int(t) for t in v.split()]
    return out


def pin_fig1_example(o):
    """Sec. 4.1-4.2 worked example (Fig. 1 text): 5x5 grid, 1-based."""
    g = _read_golden("fig1_5x5_levels.txt")
    nx, ny = g["grid"]
    T = W.laplacian_triangle((nx, ny))
    level, nlev = o.levels_row(T.row_ptr, T.col_idx)
    assert nlev == g["nlev"][0]
    ilev, jlev = o.level_sets(level, nlev)
    lev5 = sorted(int(r) + 1 for r in jlev[ilev[4]:ilev[5]])   # 1-based level 5 = index 4
    assert lev5 == g["level5_nodes"], lev5
    for node, key in ((10, "deps_of_10"), (14, "deps_of_14")):
        i = node - 1
        cols = T.col_idx[T.row_ptr[i]:T.row_ptr[i + 1]]
        deps = sorted(int(c) + 1 for c in cols if c != i)
        assert deps == g[key], (node, deps)
        # and the node sits one level above its deps
        assert all(level[i] == level[d - 1] + 1 for d in deps)


def _longest_path_levels(dense_pattern, upper):
    """Brute force: the level of i is the number of edges on the longest
    dependency chain ending at i, found by enumerating every chain."""
    n = dense_pattern.shape[0]
    deps = [[j for j in range(n) if j != i and dense_pattern[i, j]] for i in range(n)]

    def longest(i):
        best = 0
        for j in deps[i]:
            best = max(best, 1 + longest(j))
        return best
    return np.array([longest(i) for i in range(n)], dtype=np.int32)


def pin_levels_bruteforce(o):
    """Levels equal the longest dependency chain (DAG view, Sec. 4.1) on
    random tiny triangles, stored rows in random order."""
    for seed in range(12):
        n = 1 + seed % 12
        for upper in (False, True):
            T = W.random_triangle(n, seed, density=0.45, upper=upper, shuffle_rows=True)
            want = _longest_path_levels(T.dense() != 0, upper)
            for fn in (o.levels_row, o.levels_col):
                level, nlev = fn(T.row_ptr, T.col_idx, upper)
                assert np.array_equal(level, want), (seed, upper, fn.__name__, level, want)
                assert nlev == int(want.max()) + 1


def pin_levels_special(o):
    """Sec. 4.1 extremes: diagonal matrix nlev = 1, a chain nlev = n."""
    D = W.diagonal_matrix(np.arange(1, 8, dtype=float))
    level, nlev = o.levels_row(D.row_ptr, D.col_idx)
    assert nlev == 1 and not level.any()
    for upper in (False, True):
        C = W.bidiagonal(9, 2.0, 1.0, upper=upper)
        level, nlev = o.levels_row(C.row_ptr, C.col_idx, upper)
        assert nlev == 9
        assert np.array_equal(level, (np.arange(9)[::-1] if upper else np.arange(9)))


def pin_level_sets(o):
    """jlev is a permutation in nondecreasing level order, ties in ascending
    row order (numpy's stable argsort), ilev the level boundaries."""
    rng = np.random.Generator(np.random.PCG64(7))
    for n in (1, 5, 40, 300):
        nlev = 1 + int(rng.integers(0, 8))
        level = rng.integers(0, nlev, n).astype(np.int32)
        level[rng.integers(0, n)] = nlev - 1
        present = np.unique(level)
        remap = np.full(nlev, -1)
        remap[present] = np.arange(present.size)
        level = remap[level].astype(np.int32)        # every level non-empty
        nlev = present.size
        ilev, jlev = o.level_sets(level, nlev)
        assert np.array_equal(jlev, np.argsort(level, kind="stable"))
        assert ilev[0] == 0 and ilev[-1] == n
        for m in range(nlev):
            assert np.all(level[jlev[ilev[m]:ilev[m + 1]]] == m)
    # on a real triangle: the level of each listed unknown never decreases
    T = W.laplacian_triangle((6, 5, 3))
    level, nlev = o.levels_row(T.row_ptr, T.col_idx)
    ilev, jlev = o.level_sets(level, nlev)
    assert np.all(np.diff(level[jlev]) >= 0)
    assert np.array_equal(np.sort(jlev), np.arange(T.n))


def pin_depcnt(o):
    """Sec. 4.4: dependency count = stored off-diagonals of the row; for a
    Laplacian lower triangle it is the number of lower grid neighbours."""
    dims = (4, 3, 5)
    T = W.laplacian_triangle(dims)
    idx = np.arange(T.n)
    want = (idx % 4 > 0).astype(int) + ((idx // 4) % 3 > 0) + (idx // 12 > 0)
    assert np.array_equal(o.depcnt(T.row_ptr, T.col_idx), want)
    D = W.diagonal_matrix(np.ones(5))
    assert not o.depcnt(D.row_ptr, D.col_idx).any()


def _tri_dense(T):
    M = T.dense()
    if T.unit_diag:
        np.fill_diagonal(M, 1.0)
    return M


def pin_solve_dense(o):
    """Sec. 3.1/3.2 substitution vs a dense triangular solve (LAPACK)."""
    for seed in range(16):
        n = [1, 2, 3, 7, 20, 60][seed % 6]
        upper = bool(seed % 2)
        unit = seed % 4 == 3
        T = W.random_triangle(n, 100 + seed, density=0.4, upper=upper, unit_diag=unit,
                              shuffle_rows=True)
        b = W.uniform_vector(n, 200 + seed)
        x = o.solve(T.row_ptr, T.col_idx, T.vals, b, upper, unit)
        want = sla.solve_triangular(_tri_dense(T), b, lower=not upper, unit_diagonal=unit)
        assert np.allclose(x, want, rtol=1e-12, atol=1e-13 * np.abs(want).max()), (seed,)
        xc = o.solve_col(*o.transpose(T.row_ptr, T.col_idx, T.vals), b, upper, unit)
        assert np.allclose(xc, want, rtol=1e-12, atol=1e-13 * np.abs(want).max()), (seed, "col")


def pin_solve_exact_cases(o):
    """Cases with an exactly representable answer, compared bit for bit:
    diagonal x = b/d (one correctly rounded division); I - S gives prefix
    sums of integers; bidiagonal (2, -1) with b = e_0 gives x_i = 2^-(i+1)."""
    d = np.array([3.0, -7.0, 0.1, 1e300, 5e-300, 9.0])
    b = np.array([1.0, 2.0, 3.0, -4.0, 1e-10, 0.0])
    D = W.diagonal_matrix(d)
    assert np.array_equal(o.solve(D.row_ptr, D.col_idx, D.vals, b), b / d)
    n = 200
    rng = np.random.Generator(np.random.PCG64(11))
    bi = rng.integers(-1000, 1000, n).astype(float)
    for upper in (False, True):
        P = W.bidiagonal(n, 1.0, 1.0, upper=upper)
        want = np.cumsum(bi[::-1])[::-1] if upper else np.cumsum(bi)
        assert np.array_equal(o.solve(P.row_ptr, P.col_idx, P.vals, bi, upper), want)
        assert np.array_equal(o.solve(P.row_ptr, P.col_idx, P.vals, bi, upper, True), want)
        B = W.bidiagonal(60, 2.0, 1.0, upper=upper)
        e = np.zeros(60)
        e[-1 if upper else 0] = 1.0
        x = o.solve(B.row_ptr, B.col_idx, B.vals, e, upper)
        pw = 2.0 ** -(np.arange(60) + 1.0)
        assert np.array_equal(x, pw[::-1] if upper else pw)


def pin_backward_error(o):
    """Backward stability of substitution (Higham, Accuracy and Stability of
    Numerical Algorithms, Thm 8.5): |b - T x^|_i <= gamma_{m_i} (|T||x^|)_i
    with m_i the entries of row i; residual in extended precision."""
    cases = [W.laplacian_triangle((6, 7, 5)), W.laplacian_triangle((9, 8), upper=True),
             W.powerlaw_lower(3000, 5, window=500), W.ilu0_lower((7, 6, 5))]
    for T in cases:
        b = W.uniform_vector(T.n, 31)
        x = o.solve(T.row_ptr, T.col_idx, T.vals, b, T.upper)
        rows = np.repeat(np.arange(T.n), np.diff(T.row_ptr))
        v = T.vals.astype(np.longdouble)
        xl = x.astype(np.longdouble)
        r = b.astype(np.longdouble).copy()
        np.subtract.at(r, rows, v * xl[T.col_idx])
        s = np.zeros(T.n, dtype=np.longdouble)
        np.add.at(s, rows, np.abs(v * xl[T.col_idx]))
        m = np.diff(T.row_ptr).astype(float)
        gam = m * U64 / (1 - m * U64)
        assert np.all(np.abs(r) <= gam * s * 1.0000001 + 1e-300), T.name


def pin_planted(o):
    for T, xs, b in [W.c1_lap2d_64(), W.c2_lap3d(side=12), W.c2_lap3d(side=10, upper=True)]:
        x = o.solve(T.row_ptr, T.col_idx, T.vals, b, T.upper)
        assert np.abs(x - xs).max() <= 1e-13 * np.abs(xs).max(), T.name


def pin_transpose(o):
    """CSR of T^T (Sec. 3, the CSC of T) vs the dense transpose, and the
    transposed solve vs a dense solve with T^T."""
    for seed in range(8):
        n = [3, 9, 30, 50][seed % 4]
        upper = bool(seed % 2)
        unit = seed % 3 == 2
        T = W.random_triangle(n, 300 + seed, density=0.35, upper=upper, unit_diag=unit,
                              shuffle_rows=True)
        rT, cT, vT = o.transpose(T.row_ptr, T.col_idx, T.vals)
        Tt = W.Triangle(n, rT, cT, vT)
        assert np.array_equal(Tt.dense(), T.dense().T)
        g = W.uniform_vector(n, 400 + seed)
        y = o.solve_transpose(T.row_ptr, T.col_idx, T.vals, g, upper, unit)
        want = sla.solve_triangular(_tri_dense(T).T, g, lower=upper, unit_diagonal=unit)
        assert np.allclose(y, want, rtol=1e-12, atol=1e-13 * np.abs(want).max()), seed
        y2 = o.solve(rT, cT, vT, g, not upper, unit)     # second route: explicit T^T
        assert np.allclose(y, y2, rtol=1e-12, atol=1e-13 * np.abs(want).max())


def pin_multi(o):
    T = W.random_triangle(40, 77, density=0.3)
    F = np.stack([W.uniform_vector(40, s) for s in range(5)], 1)
    X = o.solve_multi(T.row_ptr, T.col_idx, T.vals, F)
    want = sla.solve_triangular(T.dense(), F, lower=True)
    assert np.allclose(X, want, rtol=1e-12, atol=1e-13)


def pin_adjoint(o):
    """Adjoint of x = T^{-1} b: dense reference gradient (grad_b = T^{-T} g,
    grad_T = -grad_b x^T on the pattern) and central finite differences of
    the loss <w, x> in the values and the right-hand side."""
    for T in [W.ilu0_lower((4, 3, 3)), W.random_triangle(25, 9, density=0.3, upper=True),
              W.random_triangle(18, 10, density=0.4, unit_diag=True)]:
        b = W.uniform_vector(T.n, 1)
        w = W.uniform_vector(T.n, 2)
        x, gb, gv = o.adjoint(T.row_ptr, T.col_idx, T.vals, b, w, T.upper, T.unit_diag)
        M = _tri_dense(T)
        gb_d = np.linalg.solve(M.T, w)
        assert np.allclose(gb, gb_d, rtol=1e-10, atol=1e-12)
        rows = np.repeat(np.arange(T.n), np.diff(T.row_ptr))
        gv_d = -gb_d[rows] * x[T.col_idx]
        if T.unit_diag:
            gv_d[T.col_idx == rows] = 0.0
        assert np.allclose(gv, gv_d, rtol=1e-10, atol=1e-12)
        rng = np.random.Generator(np.random.PCG64(3))
        h = 1e-6
        for _ in range(3):
            dv = rng.uniform(-1, 1, T.nnz)
            db = rng.uniform(-1, 1, T.n)
            lp = w @ o.solve(T.row_ptr, T.col_idx, T.vals + h * dv, b + h * db, T.upper, T.unit_diag)
            lm = w @ o.solve(T.row_ptr, T.col_idx, T.vals - h * dv, b - h * db, T.upper, T.unit_diag)
            fd = (lp - lm) / (2 * h)
            an = gv @ dv + gb @ db
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (T.name, fd, an)


def pin_validate(o):
    """Sec. 3 eq. (1) preconditions; codes by name."""
    import oracle as O
    T = W.laplacian_triangle((3, 3))
    rp, ci, v = T.row_ptr.copy(), T.col_idx.copy(), T.vals.copy()
    assert o.validate(rp, ci, v) == O.OK
    assert o.validate(rp, ci, v, upper=True) == O.NOT_TRIANGULAR
    Tu = W.laplacian_triangle((3, 3), upper=True)
    assert o.validate(Tu.row_ptr, Tu.col_idx, Tu.vals, upper=True) == O.OK
    assert o.validate(Tu.row_ptr, Tu.col_idx, Tu.vals, upper=False) == O.NOT_TRIANGULAR
    bad = rp.copy(); bad[3], bad[4] = bad[4], bad[3]
    assert o.validate(bad, ci, v) == O.BAD_ROWPTR
    bad = ci.copy(); bad[0] = 9
    assert o.validate(rp, bad, v) == O.BAD_COLIDX
    bad = ci.copy(); bad[2] = bad[1]                  # row 1: (0, 0) duplicated
    assert o.validate(rp, bad, v) == O.DUPLICATE
    vz = v.copy(); vz[0] = 0.0
    assert o.validate(rp, ci, vz) == O.ZERO_PIVOT
    assert o.validate(rp, ci, vz, unit_diag=True) == O.OK
    # drop the diagonal of row 0
    rp2 = rp.copy(); rp2[1:] -= 1
    assert o.validate(rp2, ci[1:], v[1:]) == O.MISSING_DIAG
    assert o.validate(rp2, ci[1:], v[1:], unit_diag=True) == O.OK


ALL_PINS = [pin_levels_closed_form, pin_levels_stencil9_27, pin_fig1_example, pin_levels_bruteforce, pin_levels_special,
            pin_level_sets, pin_depcnt, pin_solve_dense, pin_solve_exact_cases,
            pin_backward_error, pin_planted, pin_transpose, pin_multi, pin_adjoint, pin_validate]
