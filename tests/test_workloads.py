"""Input generators: sizes, structure and the ILU(0) factors."""
import numpy as np
import pytest

import workloads as W


def _ilu0_dense(A):
    """ILU(0), IKJ form (Saad, Iterative Methods for Sparse Linear Systems,
    Alg. 10.4), restricted to the pattern of A; returns (unit L, U)."""
    A = A.copy()
    n = A.shape[0]
    pat = A != 0
    for i in range(1, n):
        for k in range(i):
            if not pat[i, k]:
                continue
            A[i, k] /= A[k, k]
            for j in range(k + 1, n):
                if pat[i, j] and pat[k, j]:
                    A[i, j] -= A[i, k] * A[k, j]
    L = np.tril(A, -1) + np.eye(n)
    U = np.triu(A)
    return L, U


@pytest.mark.parametrize("dims", [(5, 4), (4, 3, 3), (1, 6), (3, 1, 2)])
def test_ilu0_matches_bruteforce(dims):
    Lt = W.laplacian_triangle(dims)
    Ut = W.laplacian_triangle(dims, upper=True)
    A = Lt.dense() + Ut.dense() - np.diag(np.diag(Lt.dense()))
    L, U = _ilu0_dense(A)
    T = W.ilu0_lower(dims)
    assert np.allclose(T.dense(), L, rtol=1e-14, atol=1e-15)
    assert np.allclose(T.meta["pivots"], np.diag(U), rtol=1e-14)
    # ILU(0)'s U keeps A's upper off-diagonals
    assert np.allclose(np.triu(U, 1), np.triu(A, 1))


@pytest.mark.parametrize("dims", [(64, 64), (7, 5), (128, 128, 128), (96, 96, 96), (16, 16, 16)])
def test_laplacian_sizes(dims):
    n = int(np.prod(dims))
    T = W.laplacian_triangle(dims)
    # each grid edge appears once in the lower triangle, plus n diagonals
    edges = sum((dims[a] - 1) * n // dims[a] for a in range(len(dims)))
    assert T.n == n and T.nnz == n + edges
    assert T.row_ptr.dtype == np.int32 and T.col_idx.dtype == np.int32
    U = W.laplacian_triangle(dims, upper=True)
    assert U.nnz == T.nnz
    # columns ascending in every row, diagonal last (lower) / first (upper)
    for tri, pos in ((T, -1), (U, 0)):
        r = np.arange(n)
        last = tri.row_ptr[1:] - 1 if pos == -1 else tri.row_ptr[:-1]
        assert np.array_equal(tri.col_idx[last], r)


def test_config_sizes():
    T, xs, b = W.c1_lap2d_64()
    assert (T.n, T.nnz) == (4096, 12160)
    assert np.abs(xs).max() <= 1.0
    T = W.ilu0_lower((16, 16, 16))
    assert (T.n, T.nnz) == (4096, 15616)


def test_powerlaw_structure():
    T = W.powerlaw_lower(60000, 3, window=5000)
    k = np.diff(T.row_ptr) - 1
    rows = np.repeat(np.arange(T.n), np.diff(T.row_ptr))
    assert np.all(T.col_idx <= rows)
    assert np.all(T.col_idx[T.row_ptr[1:] - 1] == np.arange(T.n))    # diagonal last
    off = T.col_idx != rows
    assert np.all(rows[off] - T.col_idx[off] <= 5000)
    # strictly ascending columns within a row (no duplicates)
    same_row = rows[1:] == rows[:-1]
    assert np.all(np.diff(T.col_idx)[same_row] > 0)
    assert 7.0 < k[1000:].mean() < 9.0 and k.max() <= 2000
    d = T.vals[~off]
    assert d.min() >= 1.0 and d.max() <= 2.0
    assert np.all(np.abs(T.vals[off]) <= 1.0 / k[rows[off]])


def test_block_diagonal():
    tris = [W.ilu0_lower((s, s)) for s in (3, 5, 4)]
    B = W.concat_block_diagonal(tris)
    D = B.dense()
    off = 0
    for t in tris:
        assert np.array_equal(D[off:off + t.n, off:off + t.n], t.dense())
        off += t.n
    assert B.nnz == sum(t.nnz for t in tris)


def test_planted_rhs():
    T = W.laplacian_triangle((6, 5))
    xs, b = W.planted(T, 9)
    assert np.allclose(T.dense() @ xs, b, rtol=1e-15, atol=1e-15)
    X, B = W.planted(T, 9, nrhs=3)
    assert X.shape == (30, 3) and np.allclose(T.dense() @ X, B)
