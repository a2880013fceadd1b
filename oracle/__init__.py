"""CPU oracle for sparse triangular solves (arXiv:1710.04985).

TEST INFRASTRUCTURE ONLY.  The oracle is the checker: only the test suite,
the smoke check and the CPU-baseline leg of the benchmark may import it.  The
HIP library never links, imports or calls it, and the two share no code.

The arithmetic lives in ``sptrsv_oracle.c`` (plain C, FP64, one thread), which
is compiled here with ``gcc -O2`` into ``oracle/_build/liboracle.so``.  This
module only marshals numpy arrays into it.  Each wrapper names the passage of
the paper its C function follows.

Parity status: every function below is pinned by CPU tests against values the
paper or the mathematics fixes (closed forms, the worked 5x5 example, dense
solves, brute force on tiny inputs, finite differences).  None is unpinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sptrsv_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")

# oracle status codes (mirror of the #defines in sptrsv_oracle.c)
OK = 0
INVALID_ARG = -1
BAD_ROWPTR = -2
BAD_COLIDX = -3
NOT_TRIANGULAR = -4
DUPLICATE = -5
MISSING_DIAG = -6
ZERO_PIVOT = -7

_lock = threading.Lock()
_lib = None


def compile_oracle(src: str = _SRC, out: str = _LIB_PATH, extra_flags=()) -> str:
    """Compile the C oracle into a shared library; returns its path."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", *extra_flags, src, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_I32P = ctypes.POINTER(ctypes.c_int32)
_F64P = ctypes.POINTER(ctypes.c_double)


def _declare(lib):
    i, p, d = ctypes.c_int, _I32P, _F64P
    sig = {
        "oracle_validate": (i, [i, i, p, p, d, i, i]),
        "oracle_levels_row": (i, [i, p, p, i, p]),
        "oracle_levels_col": (i, [i, p, p, i, p]),
        "oracle_transpose": (None, [i, p, p, d, p, p, d]),
        "oracle_level_sets": (None, [i, p, i, p, p]),
        "oracle_depcnt": (None, [i, p, p, p]),
        "oracle_solve_row": (i, [i, p, p, d, i, i, d, d]),
        "oracle_solve_col": (i, [i, p, p, d, i, i, d, d]),
        "oracle_solve_transpose": (i, [i, p, p, d, i, i, d, d]),
        "oracle_solve_multi": (i, [i, p, p, d, i, i, i, i, d, d]),
        "oracle_grad_vals": (None, [i, p, p, i, d, d, d]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load_library(path: str | None = None):
    """Load (building if needed) the oracle library.  A different path loads
    a separate copy (used by the mutation tests)."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            stale = (not os.path.exists(_LIB_PATH)
                     or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC))
            if stale:
                compile_oracle()
            _lib = _declare(ctypes.CDLL(_LIB_PATH))
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I32P)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_F64P)


def _null_f64():
    return ctypes.cast(None, _F64P)


class Oracle:
    """Thin numpy front end over one copy of the C oracle."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else load_library()

    # Sec. 3, eq. (1): problem statement
    def validate(self, row_ptr, col_idx, vals, upper=False, unit_diag=False):
        rp, rpp = _i32(row_ptr)
        ci, cip = _i32(col_idx)
        n = len(rp) - 1
        if vals is None:
            vp = _null_f64()
        else:
            v, vp = _f64(vals)
        return self.lib.oracle_validate(n, len(ci), rpp, cip, vp, int(upper), int(unit_diag))

    # Sec. 4.1, row-wise level formula
    def levels_row(self, row_ptr, col_idx, upper=False):
        rp, rpp = _i32(row_ptr)
        ci, cip = _i32(col_idx)
        n = len(rp) - 1
        level = np.zeros(n, dtype=np.int32)
        nlev = self.lib.oracle_levels_row(n, rpp, cip, int(upper), level.ctypes.data_as(_I32P))
        return level, nlev

    # Sec. 4.1, column-wise level formula
    def levels_col(self, row_ptr, col_idx, upper=False):
        rp, rpp = _i32(row_ptr)
        ci, cip = _i32(col_idx)
        n = len(rp) - 1
        level = np.zeros(n, dtype=np.int32)
        nlev = self.lib.oracle_levels_col(n, rpp, cip, int(upper), level.ctypes.data_as(_I32P))
        return level, nlev

    # Sec. 3: CSR of T^T == CSC of T
    def transpose(self, row_ptr, col_idx, vals=None):
        rp, rpp = _i32(row_ptr)
        ci, cip = _i32(col_idx)
        n = len(rp) - 1
        rowT = np.zeros(n + 1, dtype=np.int32)
        colT = np.zeros(len(ci), dtype=np.int32)
        if vals is None:
            vp, valsT, vtp = _null_f64(), None, _null_f64()
        else:
            v, vp = _f64(vals)
            valsT = np.zeros(len(ci), dtype=np.float64)
            vtp = valsT.ctypes.data_as(_F64P)
        self.lib.oracle_transpose(n, rpp, cip, vp, rowT.ctypes.data_as(_I32P),
                                  colT.ctypes.data_as(_I32P), vtp)
        return rowT, colT, valsT

    # Sec. 4.1: jlev / ilev
    def level_sets(self, level, nlev):
        lv, lvp = _i32(level)
        n = len(lv)
        ilev = np.zeros(nlev + 1, dtype=np.int32)
        jlev = np.zeros(n, dtype=np.int32)
        self.lib.oracle_level_sets(n, lvp, int(nlev), ilev.ctypes.data_as(_I32P),
                                   jlev.ctypes.data_as(_I32P))
        return ilev, jlev

    # Sec. 4.4: dependency counts
    def depcnt(self, row_ptr, col_idx):
        rp, rpp = _i32(row_ptr)
        ci, cip = _i32(col_idx)
        n = len(rp) - 1
        dc = np.zeros(n, dtype=np.int32)
        self.lib.oracle_depcnt(n, rpp, cip, dc.ctypes.data_as(_I32P))
        return dc

    def analyze(self, row_ptr, col_idx, upper=False):
        """level, nlev, ilev, jlev, depcnt of one triangle."""
        level, nlev = self.levels_row(row_ptr, col_idx, upper)
        ilev, jlev = self.level_sets(level, nlev)
        return level, nlev, ilev, jlev, self.depcnt(row_ptr, col_idx)

    def _check(self, st):
        if st != OK:
            raise ValueError("oracle status %d" % st)

    # Sec. 3.1 / 3.2: row-wise forward / backward substitution
    def solve(self, row_ptr, col_idx, vals, f, upper=False, unit_diag=False):
        rp, rpp = _i32(row_ptr)
        ci, cip = _i32(col_idx)
        v, vp = _f64(vals)
        fb, fp = _f64(f)
        n = len(rp) - 1
        x = np.zeros(n, dtype=np.float64)
        self._check(self.lib.oracle_solve_row(n, rpp, cip, vp, int(upper), int(unit_diag),
                                              fp, x.ctypes.data_as(_F64P)))
        return x

    # Sec. 3.2: column-wise substitution on a CSC triangle
    def solve_col(self, ib, jb, bv, f, upper=False, unit_diag=False):
        ibb, ibp = _i32(ib)
        jbb, jbp = _i32(jb)
        v, vp = _f64(bv)
        fb, fp = _f64(f)
        n = len(ibb) - 1
        x = np.zeros(n, dtype=np.float64)
        self._check(self.lib.oracle_solve_col(n, ibp, jbp, vp, int(upper), int(unit_diag),
                                              fp, x.ctypes.data_as(_F64P)))
        return x

    # Sec. 3.2 column sweep read on T's CSR: T^T y = g
    def solve_transpose(self, row_ptr, col_idx, vals, g, upper=False, unit_diag=False):
        rp, rpp = _i32(row_ptr)
        ci, cip = _i32(col_idx)
        v, vp = _f64(vals)
        gb, gp = _f64(g)
        n = len(rp) - 1
        y = np.zeros(n, dtype=np.float64)
        self._check(self.lib.oracle_solve_transpose(n, rpp, cip, vp, int(upper), int(unit_diag),
                                                    gp, y.ctypes.data_as(_F64P)))
        return y

    def solve_multi(self, row_ptr, col_idx, vals, F, upper=False, unit_diag=False):
        """F: (n, nrhs) array; solved column by column (column-major, ld=n)."""
        rp, rpp = _i32(row_ptr)
        ci, cip = _i32(col_idx)
        v, vp = _f64(vals)
        n = len(rp) - 1
        F = np.asarray(F, dtype=np.float64)
        nrhs = F.shape[1]
        Fc = np.asfortranarray(F)
        X = np.zeros((n, nrhs), dtype=np.float64, order="F")
        self._check(self.lib.oracle_solve_multi(n, rpp, cip, vp, int(upper), int(unit_diag),
                                                nrhs, n, Fc.ctypes.data_as(_F64P),
                                                X.ctypes.data_as(_F64P)))
        return X

    def solve_batched(self, systems, fs, upper=False, unit_diag=False):
        """One substitution per independent system: systems = [(rp, ci, vals)]."""
        return [self.solve(rp, ci, v, f, upper, unit_diag) for (rp, ci, v), f in zip(systems, fs)]

    def grad_vals(self, row_ptr, col_idx, grad_f, x, unit_diag=False):
        rp, rpp = _i32(row_ptr)
        ci, cip = _i32(col_idx)
        gf, gfp = _f64(grad_f)
        xx, xp = _f64(x)
        n = len(rp) - 1
        gv = np.zeros(len(ci), dtype=np.float64)
        self.lib.oracle_grad_vals(n, rpp, cip, int(unit_diag), gfp, xp, gv.ctypes.data_as(_F64P))
        return gv

    def adjoint(self, row_ptr, col_idx, vals, f, grad_x, upper=False, unit_diag=False):
        """Forward x = T^{-1} f and the adjoint (grad_f, grad_vals)."""
        x = self.solve(row_ptr, col_idx, vals, f, upper, unit_diag)
        grad_f = self.solve_transpose(row_ptr, col_idx, vals, grad_x, upper, unit_diag)
        return x, grad_f, self.grad_vals(row_ptr, col_idx, grad_f, x, unit_diag)


_default = None


def get() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default
