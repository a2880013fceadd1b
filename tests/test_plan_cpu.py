"""Level-ordered layout and work chunks of the library's host analysis,
checked on the CPU (the kernels index b, x and the matrix through them)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1710_04985_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    out = tmp_path_factory.mktemp("plan") / "plan_check.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-I", CSRC,
                    os.path.join(ROOT, "tests", "cpp", "plan_check.cpp"),
                    os.path.join(CSRC, "analysis.cpp"), "-o", str(out)], check=True)
    lib = ctypes.CDLL(str(out))
    P = ctypes.POINTER(ctypes.c_int32)
    lib.check_plan.argtypes = [ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, ctypes.c_int]
    return lib


def _tris():
    return [W.laplacian_triangle((9, 7, 5)), W.laplacian_triangle((9, 7, 5), upper=True),
            W.laplacian_triangle((64, 64)), W.powerlaw_lower(30000, 11, window=2000),
            W.random_triangle(80, 3, density=0.5, upper=True, shuffle_rows=True),
            W.diagonal_matrix(np.ones(100)), W.bidiagonal_fast(300, 2.0, 1.0),
            W.ilu0_lower((6, 5, 4))]


@pytest.mark.parametrize("T", _tris(), ids=lambda t: t.name)
@pytest.mark.parametrize("policy", [(0, 1, 0, 1), (0, 4, 0, 4), (0, 8, 0, 2), (1, 4, 0, 1),
                                    (1, 4, 0, 4), (1, 1, 0, 3), (4, 4, 0, 4), (64, 4, 0, 4),
                                    (0, 4, 4, 4), (0, 4, 1, 1), (0, 4, 64, 2)])
def test_plan_and_chunks(checker, T, policy):
    rp = np.ascontiguousarray(T.row_ptr, np.int32)
    ci = np.ascontiguousarray(T.col_idx, np.int32)
    P = ctypes.POINTER(ctypes.c_int32)
    for unit in (0, 1):
        rc = checker.check_plan(T.n, rp.ctypes.data_as(P), ci.ctypes.data_as(P), int(T.upper),
                                unit, *policy)
        assert rc == 0, "invariant %d violated" % rc


def _concat(tris):
    """Block-diagonal concatenation of lower/upper triangles of one kind."""
    rps, cis, row0 = [np.zeros(1, np.int64)], [], [0]
    off = nnz = 0
    for t in tris:
        rps.append(np.asarray(t.row_ptr[1:], np.int64) + nnz)
        cis.append(np.asarray(t.col_idx, np.int64) + off)
        off += t.n
        nnz += t.nnz
        row0.append(off)
    return (off, np.ascontiguousarray(np.concatenate(rps), np.int32),
            np.ascontiguousarray(np.concatenate(cis), np.int32), np.asarray(row0, np.int32))


@pytest.mark.parametrize("case", ["c1", "batch_lower", "batch_upper", "one_row_systems",
                                  "too_many_rows"])
def test_block_resident_layout(checker, case):
    """The resident block kernel's LDS layout and level loop, modelled on the
    CPU with every access bounds-checked, against plain substitution."""
    P = ctypes.POINTER(ctypes.c_int32)
    checker.check_block_resident.argtypes = [ctypes.c_int, P, P, ctypes.c_int, ctypes.c_int, P,
                                             ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_longlong)]
    if case == "c1":
        tris = [W.laplacian_triangle((64, 64))]
    elif case == "batch_lower":
        tris = [W.ilu0_lower((9, 9)), W.laplacian_triangle((5, 4, 3)), W.ilu0_lower((14, 6)),
                W.random_triangle(40, 7, density=0.2, shuffle_rows=True)]
    elif case == "batch_upper":
        tris = [W.laplacian_triangle((6, 5), upper=True), W.laplacian_triangle((4, 4, 4), upper=True)]
    elif case == "one_row_systems":
        tris = [W.diagonal_matrix(np.ones(1)), W.bidiagonal_fast(5, 2.0, 1.0),
                W.diagonal_matrix(np.ones(3))]
    else:
        tris = [W.laplacian_triangle((260, 260))]
    n, rp, ci, row0 = _concat(tris)
    upper = int(tris[0].upper)
    for vb, tiny in ((8, 0), (4, 0), (8, 1)):
        nbytes = ctypes.c_longlong(0)
        rc = checker.check_block_resident(n, rp.ctypes.data_as(P), ci.ctypes.data_as(P), upper,
                                          len(tris), row0.ctypes.data_as(P), vb, tiny,
                                          ctypes.byref(nbytes))
        assert rc == 0, "check %d violated (vb %d, tiny %d)" % (rc, vb, tiny)
        if case == "c1":
            # 4096 rows, 8064 off-diagonals, 127 levels
            # (one dummy entry and one zero slot of x on top)
            assert nbytes.value == vb * (2 * 4096 + 8064 + 2) + 2 * 4097 + 2 * 8065 + 2 * 128
            assert nbytes.value <= 160 * 1024
        elif case == "too_many_rows":
            assert nbytes.value == -1
        else:
            assert nbytes.value > 0
