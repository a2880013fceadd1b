"""Seeded synthetic inputs for sparse triangular solves.

This module only builds inputs: CSR triangles of the paper's model problems
(2-D 5-point and 3-D 7-point Laplacians in lexicographic order, Sec. 5.1),
ILU(0) factors of those Laplacians, random power-law triangles standing in
for the paper's general matrices (Sec. 5.2, Table 3, which are not used
here), planted solutions and right-hand sides.  It contains no part of the
triangular-solve method itself and is shared by the oracle tests, the GPU
tests and the benchmark.

Storage convention: CSR with int32 indices, columns ascending inside a row,
the diagonal stored inside the row (last in a lower row, first in an upper
row).  Grid index i = ix + nx*iy + nx*ny*iz (x fastest).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class Triangle:
    n: int
    row_ptr: np.ndarray          # int32[n+1]
    col_idx: np.ndarray          # int32[nnz]
    vals: np.ndarray             # float64[nnz]
    upper: bool = False
    unit_diag: bool = False
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self):
        return sp.csr_matrix((self.vals, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def dense(self):
        return self.scipy().toarray()

    def matvec(self, x):
        """b = T x, accumulated in FP64 in row order (scipy's CSR kernel).
        Under unit_diag the stored diagonal is replaced by 1."""
        if not self.unit_diag:
            return self.scipy() @ np.asarray(x, dtype=np.float64)
        v = self.vals.copy()
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        diag = self.col_idx == rows
        v[diag] = 0.0
        m = sp.csr_matrix((v, self.col_idx, self.row_ptr), shape=(self.n, self.n))
        return m @ np.asarray(x, dtype=np.float64) + np.asarray(x, dtype=np.float64)

    def astype_vals(self, dtype):
        return Triangle(self.n, self.row_ptr, self.col_idx, self.vals.astype(dtype),
                        self.upper, self.unit_diag, self.name, dict(self.meta))


def _assemble(cols: np.ndarray, mask: np.ndarray, vals: np.ndarray, n: int):
    """cols/mask/vals: (n, w) candidate entries per row in storage order."""
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return (row_ptr.astype(np.int32), cols[mask].astype(np.int32),
            vals[mask].astype(np.float64))


def laplacian_triangle(dims, upper=False, diag=None, off=-1.0, name="") -> Triangle:
    """Lower or upper triangle (diagonal included) of the 2-D 5-point
    (len(dims)==2) or 3-D 7-point (len(dims)==3) Laplacian, lexicographic."""
    dims = tuple(int(d) for d in dims)
    if diag is None:
        diag = 4.0 if len(dims) == 2 else 6.0
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    stride = 1
    strides = []
    rem = idx
    for d in dims:
        coords.append(rem % d)
        rem = rem // d
        strides.append(stride)
        stride *= d
    cand_c, cand_m, cand_v = [], [], []
    if not upper:
        for ax in reversed(range(len(dims))):       # farthest first -> ascending
            cand_c.append(idx - strides[ax])
            cand_m.append(coords[ax] > 0)
            cand_v.append(np.full(n, off))
        cand_c.append(idx)
        cand_m.append(np.ones(n, dtype=bool))
        cand_v.append(np.full(n, diag))
    else:
        cand_c.append(idx)
        cand_m.append(np.ones(n, dtype=bool))
        cand_v.append(np.full(n, diag))
        for ax in range(len(dims)):                  # nearest first -> ascending
            cand_c.append(idx + strides[ax])
            cand_m.append(coords[ax] < dims[ax] - 1)
            cand_v.append(np.full(n, off))
    rp, ci, v = _assemble(np.stack(cand_c, 1), np.stack(cand_m, 1), np.stack(cand_v, 1), n)
    return Triangle(n, rp, ci, v, upper=upper, name=name or
                    "lap%dd_%s_%s" % (len(dims), "x".join(map(str, dims)), "U" if upper else "L"),
                    meta={"dims": dims})


def _stencil_offsets(dims, points):
    """Neighbour offsets of the 5/9-point (2-D) or 7/27-point (3-D) stencil."""
    import itertools
    d = len(dims)
    if points in (5, 7):
        offs = []
        for ax in range(d):
            for sgn in (-1, 1):
                o = [0] * d
                o[ax] = sgn
                offs.append(tuple(o))
        return offs
    if points in (9, 27):
        return [o for o in itertools.product((-1, 0, 1), repeat=d) if any(o)]
    raise ValueError("stencil points must be 5/9 (2-D) or 7/27 (3-D)")


def stencil_triangle(dims, points, upper=False, diag=None, off=-1.0, name="") -> Triangle:
    """Lower or upper triangle (diagonal included) of a Laplacian-type stencil
    operator on a regular grid (Sec. 5.1): 5- or 9-point in 2-D, 7- or
    27-point in 3-D, lexicographic order (x fastest), off-diagonals `off`,
    diagonal `diag` (default: the number of neighbours).  An offset belongs to
    the lower triangle when its last nonzero component (z, then y, then x) is
    negative."""
    dims = tuple(int(v) for v in dims)
    offs = _stencil_offsets(dims, points)
    if diag is None:
        diag = float(len(offs))
    n = int(np.prod(dims))
    idx = np.arange(n, dtype=np.int64)
    coords, strides, stride, rem = [], [], 1, idx
    for dd in dims:
        coords.append(rem % dd)
        rem = rem // dd
        strides.append(stride)
        stride *= dd

    def is_lower(o):
        for v in reversed(o):
            if v:
                return v < 0
        return False

    sel = [o for o in offs if is_lower(o) != upper]
    # ascending column order: sort by linear offset
    sel.sort(key=lambda o: sum(v * st for v, st in zip(o, strides)))
    cand_c, cand_m, cand_v = [], [], []
    lin = [sum(v * st for v, st in zip(o, strides)) for o in sel]
    before = [o for o, l in zip(sel, lin) if l < 0]
    after = [o for o, l in zip(sel, lin) if l > 0]
    for group in (before, None, after):
        if group is None:
            cand_c.append(idx)
            cand_m.append(np.ones(n, dtype=bool))
            cand_v.append(np.full(n, diag))
            continue
        for o in group:
            m = np.ones(n, dtype=bool)
            for ax, v in enumerate(o):
                if v < 0:
                    m &= coords[ax] >= -v
                elif v > 0:
                    m &= coords[ax] < dims[ax] - v
            cand_c.append(idx + sum(v * st for v, st in zip(o, strides)))
            cand_m.append(m)
            cand_v.append(np.full(n, off))
    rp, ci, v = _assemble(np.stack(cand_c, 1), np.stack(cand_m, 1), np.stack(cand_v, 1), n)
    return Triangle(n, rp, ci, v, upper=upper,
                    name=name or "stencil%d_%s_%s" % (points, "x".join(map(str, dims)), "U" if upper else "L"),
                    meta={"dims": dims, "points": points})


# grids of the paper's Table 2 (2-D n = 2^20, 3-D n = 2^21) and their aspect ratios
TABLE2_2D = [(1024, 1024), (512, 2048), (256, 4096), (128, 8192), (64, 16384)]
TABLE2_3D = [(128, 128, 128), (64, 128, 256), (64, 64, 512), (32, 64, 1024), (32, 32, 2048)]


def ilu0_lower(dims, name="") -> Triangle:
    """Unit lower factor L of ILU(0) of the 5-point (2-D, diagonal 4) or
    7-point (3-D, diagonal 6) Laplacian with off-diagonals -1, natural order.
    For these stencils ILU(0) has no off-diagonal updates, so the pivots obey
    d_i = c - sum_{grid neighbour j < i} 1/d_j and L_ij = -1/d_j; the unit
    diagonal is stored explicitly as 1.0.  The pivots are evaluated one
    anti-diagonal (ix+iy+iz = const) at a time, each depending only on the
    previous one."""
    dims = tuple(int(d) for d in dims)
    c = 4.0 if len(dims) == 2 else 6.0
    grid = np.zeros(dims[::-1], dtype=np.float64)       # indexed [iz, iy, ix] / [iy, ix]
    mesh = np.meshgrid(*[np.arange(d) for d in dims[::-1]], indexing="ij")
    s = sum(mesh)
    for m in range(int(s.max()) + 1):
        sel = s == m
        acc = np.full(int(sel.sum()), c)
        pos = [a[sel] for a in mesh]
        for ax in range(len(dims)):
            p = [q.copy() for q in pos]
            p[ax] = p[ax] - 1
            ok = p[ax] >= 0
            if ok.any():
                nb = grid[tuple(q[ok] for q in p)]
                acc[ok] -= 1.0 / nb
        grid[sel] = acc
    dpiv = grid.reshape(-1)                                 # lexicographic, x fastest
    T = laplacian_triangle(dims, upper=False, diag=1.0, off=-1.0)
    rows = np.repeat(np.arange(T.n), np.diff(T.row_ptr))
    offd = T.col_idx != rows
    T.vals = T.vals.copy()
    T.vals[offd] = -1.0 / dpiv[T.col_idx[offd]]
    T.vals[~offd] = 1.0
    T.name = name or "ilu0L_%s" % "x".join(map(str, dims))
    T.meta["pivots"] = dpiv
    return T


POWERLAW_ALPHA = 1.85508818062782   # P(k) ~ k^-alpha on [1, 2000] has mean 8


def powerlaw_lower(n, seed, kmax=2000, window=50000, alpha=POWERLAW_ALPHA, name="") -> Triangle:
    """Random general lower triangle: off-diagonal count k_i drawn from a
    power law on [1, kmax] (mean 8), capped by the columns available;
    columns uniform without replacement in [max(0, i-window), i), sorted;
    diagonal last.  Off-diagonals U[-1,1]/k_i, diagonal U[1,2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = np.arange(1, kmax + 1, dtype=np.float64)
    w = ks ** -alpha
    cdf = np.cumsum(w) / w.sum()
    k = np.searchsorted(cdf, rng.random(n), side="right") + 1
    k = np.minimum(k, kmax)
    i = np.arange(n, dtype=np.int64)
    lo = np.maximum(0, i - window)
    avail = i - lo
    k = np.minimum(k, avail).astype(np.int64)
    # Rows whose window is not much wider than k are drawn exactly, one by one;
    # the rest are drawn with replacement and their duplicates redrawn.
    dense = np.nonzero(4 * k > avail)[0]
    rows = np.repeat(i, k)
    cols = lo[rows] + (rng.random(rows.size) * avail[rows]).astype(np.int64)
    cols = np.minimum(cols, rows - 1)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    start = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(k, out=start[1:])
    for r in dense:
        cols[start[r]:start[r + 1]] = np.sort(lo[r] + rng.choice(avail[r], k[r], replace=False))
    for _ in range(1000):
        dup = np.zeros(rows.size, dtype=bool)
        dup[1:] = (rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])
        if not dup.any():
            break
        bad = np.unique(rows[dup])
        sel = np.concatenate([np.arange(start[r], start[r + 1]) for r in bad])
        d_sel = dup[sel]
        c_sel = cols[sel]
        r_sel = rows[sel]
        c_sel[d_sel] = np.minimum(lo[r_sel[d_sel]] + (rng.random(int(d_sel.sum())) *
                                  avail[r_sel[d_sel]]).astype(np.int64), r_sel[d_sel] - 1)
        o2 = np.lexsort((c_sel, r_sel))
        cols[sel] = c_sel[o2]
    else:
        raise RuntimeError("duplicate removal did not converge")
    offv = rng.uniform(-1.0, 1.0, rows.size) / k[rows]
    dv = rng.uniform(1.0, 2.0, n)
    # interleave: off-diagonals of row i (sorted) then its diagonal
    allrows = np.concatenate([rows, i])
    allcols = np.concatenate([cols, i])
    allvals = np.concatenate([offv, dv])
    isdiag = np.concatenate([np.zeros(rows.size, bool), np.ones(n, bool)])
    order = np.lexsort((isdiag, allcols, allrows))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(k + 1, out=row_ptr[1:])
    return Triangle(n, row_ptr.astype(np.int32), allcols[order].astype(np.int32),
                    allvals[order], upper=False, name=name or "powerlaw_%d" % n,
                    meta={"seed": seed, "k": k})


def random_triangle(n, seed, density=0.3, upper=False, unit_diag=False, zero_diag_ok=False,
                    shuffle_rows=False) -> Triangle:
    """Small random triangle for dense cross-checks; row diagonally dominant.
    shuffle_rows stores each row's entries in a random order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    M = np.zeros((n, n))
    mask = rng.random((n, n)) < density
    M[mask] = rng.uniform(-1, 1, int(mask.sum()))
    M = np.triu(M, 1) if upper else np.tril(M, -1)
    rs = np.abs(M).sum(axis=1)
    d = (rs + rng.uniform(0.5, 1.5, n)) * rng.choice([-1.0, 1.0], n)
    np.fill_diagonal(M, d)
    pat = (M != 0)
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(pat.sum(1))
    cols, vals = [], []
    for r in range(n):
        c = np.nonzero(pat[r])[0]
        if shuffle_rows:
            c = rng.permutation(c)
        cols.append(c)
        vals.append(M[r, c])
    ci = np.concatenate(cols).astype(np.int32) if n else np.zeros(0, np.int32)
    v = np.concatenate(vals) if n else np.zeros(0)
    return Triangle(n, rp, ci, v, upper=upper, unit_diag=unit_diag,
                    name="rand%d_s%d" % (n, seed))


def diagonal_matrix(d) -> Triangle:
    d = np.asarray(d, dtype=np.float64)
    n = d.size
    return Triangle(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                    d.copy(), name="diag%d" % n)


def bidiagonal(n, d, c, upper=False) -> Triangle:
    """Diagonal d, the neighbouring off-diagonal -c (sub for lower, super for upper)."""
    cols, vals, rp = [], [], [0]
    for i in range(n):
        if not upper:
            if i > 0:
                cols.append(i - 1); vals.append(-c)
            cols.append(i); vals.append(d)
        else:
            cols.append(i); vals.append(d)
            if i < n - 1:
                cols.append(i + 1); vals.append(-c)
        rp.append(len(cols))
    return Triangle(n, np.array(rp, np.int32), np.array(cols, np.int32),
                    np.array(vals, np.float64), upper=upper, name="bidiag%d" % n)


def bidiagonal_fast(n, d, c, upper=False, unit_diag=False) -> Triangle:
    """Vectorised bidiagonal for large n (same layout as bidiagonal)."""
    i = np.arange(n, dtype=np.int64)
    if not upper:
        cand = np.stack([i - 1, i], 1)
        m = np.stack([i > 0, np.ones(n, bool)], 1)
        v = np.stack([np.full(n, -c), np.full(n, d)], 1)
    else:
        cand = np.stack([i, i + 1], 1)
        m = np.stack([np.ones(n, bool), i < n - 1], 1)
        v = np.stack([np.full(n, d), np.full(n, -c)], 1)
    rp, ci, vv = _assemble(cand, m, v, n)
    return Triangle(n, rp, ci, vv, upper=upper, unit_diag=unit_diag, name="bidiag%d" % n)


def planted(T: Triangle, seed, nrhs=None, dtype=np.float64):
    """x* ~ U[-1,1] (PCG64(seed)), b = T x* in FP64.  nrhs -> (n, nrhs)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if nrhs is None:
        xs = rng.uniform(-1.0, 1.0, T.n)
        return xs, T.matvec(xs)
    X = rng.uniform(-1.0, 1.0, (nrhs, T.n)).T      # column j = draw j
    B = np.stack([T.matvec(X[:, j]) for j in range(nrhs)], 1)
    return X, B


def uniform_vector(n, seed, lo=-1.0, hi=1.0):
    return np.random.Generator(np.random.PCG64(seed)).uniform(lo, hi, n)


def concat_block_diagonal(tris) -> Triangle:
    """Block-diagonal concatenation of independent triangles (same uplo)."""
    rps, cis, vs, off, nnz_off = [], [], [], 0, 0
    for t in tris:
        rps.append(t.row_ptr[:-1].astype(np.int64) + nnz_off)
        cis.append(t.col_idx.astype(np.int64) + off)
        vs.append(t.vals)
        off += t.n
        nnz_off += t.nnz
    rp = np.concatenate(rps + [np.array([nnz_off])]).astype(np.int32)
    return Triangle(off, rp, np.concatenate(cis).astype(np.int32), np.concatenate(vs),
                    upper=tris[0].upper, unit_diag=tris[0].unit_diag, name="blockdiag%d" % len(tris),
                    meta={"sizes": [t.n for t in tris]})


# ---------------------------------------------------------------------
# The five workloads (sizes of the configurations the bench and tests use)
# ---------------------------------------------------------------------

def c1_lap2d_64():
    """2-D 5-point Laplacian lower triangle, 64x64 (n 4096), seed 1."""
    T = laplacian_triangle((64, 64), upper=False, diag=4.0)
    xs, b = planted(T, 1)
    return T, xs, b


def c2_lap3d(side=128, upper=False, seed=2):
    """3-D 7-point Laplacian lower/upper triangle on side^3 (128^3: n 2,097,152)."""
    T = laplacian_triangle((side, side, side), upper=upper, diag=6.0)
    xs, b = planted(T, seed + (1 if upper else 0))
    return T, xs, b


def c3_powerlaw(n=1_000_000, seed=3):
    T = powerlaw_lower(n, seed)
    xs, b = planted(T, seed + 100)
    return T, xs, b


def c4a_sides(count=256, seed=4, lo=32, hi=256):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, count)


def c4a_batch(count=256, seed=4, lo=32, hi=256):
    """count ILU(0) unit-lower factors of 2-D 5-point Laplacians on square
    grids with side ~ U{lo..hi}; planted x* per system."""
    sides = c4a_sides(count, seed, lo, hi)
    cache = {}
    tris, xs, bs = [], [], []
    for s_i, s in enumerate(sides):
        s = int(s)
        if s not in cache:
            cache[s] = ilu0_lower((s, s))
        T = cache[s]
        x, b = planted(T, 1000 + s_i)
        tris.append(T)
        xs.append(x)
        bs.append(b)
    return tris, xs, bs


def c4b_multi(side=128, nrhs=16, seed=5):
    T = laplacian_triangle((side, side, side), upper=False, diag=6.0)
    X, B = planted(T, seed, nrhs=nrhs)
    return T, X, B


def c5_ilu3d(side=96, seed=6):
    """ILU(0) unit-lower factor of the 3-D 7-point Laplacian; b and the loss
    weight w ~ U[-1,1]."""
    T = ilu0_lower((side, side, side))
    xs, b = planted(T, seed)
    w = uniform_vector(T.n, seed + 100)
    return T, b, w
