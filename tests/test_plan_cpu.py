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
