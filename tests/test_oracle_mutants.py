"""Planted mistakes in the oracle must be caught by its pins.

Each case copies oracle/sptrsv_oracle.c, replaces one fragment with a
plausible mistake (a dropped term, a wrong sign or index, a transposed
operand, a reversed sweep), compiles the copy on the CPU and runs every pin
against it: at least one pin has to fail.  The real oracle is never touched.
"""
import os

import pytest

import oracle
from pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "sptrsv_oracle.c")

MUTANTS = [
    # levels, row formula
    ("level_drop_plus1", "if (level[j] + 1 > lev) lev = level[j] + 1;", "if (level[j] > lev) lev = level[j];"),
    ("level_upper_sweep_forward", "int i = upper ? (n - 1 - t) : t;\n        int lev", "int i = t;\n        int lev"),
    ("level_counts_diag", "if (j == i) continue;\n            if (level[j]", "if (j > i) continue;\n            if (level[j]"),
    ("level_nlev_off_by_one", "if (lev + 1 > nlev) nlev = lev + 1;", "if (lev > nlev) nlev = lev;"),
    # levels, column formula
    ("levcol_wrong_target", "if (level[j] + 1 > level[i]) level[i] = level[j] + 1;",
     "if (level[i] + 1 > level[j]) level[j] = level[i] + 1;"),
    ("levcol_upper_sweep", "int j = upper ? (n - 1 - t) : t;       /* column j */", "int j = t;"),
    # level sets
    ("levelsets_no_scan", "for (int m = 0; m < nlev; m++) ilev[m + 1] += ilev[m];", ""),
    ("levelsets_reverse_rows", "for (int i = 0; i < n; i++) jlev[next[level[i]]++] = i;",
     "for (int i = n - 1; i >= 0; i--) jlev[next[level[i]]++] = i;"),
    # dependency counts
    ("depcnt_counts_diag", "if (col_idx[k] != i) c++;", "c++;"),
    # row-wise substitution
    ("solve_sign", "xi = xi - vals[k] * x[j];", "xi = xi + vals[k] * x[j];"),
    ("solve_wrong_index", "xi = xi - vals[k] * x[j];", "xi = xi - vals[k] * x[i];"),
    ("solve_multiply_by_d", "xi = xi / d;", "xi = xi * d;"),
    ("solve_drop_divide", "xi = xi / d;", ";"),
    ("solve_upper_forward", "int i = upper ? (n - 1 - t) : t;\n        double xi", "int i = t;\n        double xi"),
    ("solve_unit_ignored", "if (!unit_diag) {\n            if (!have_d || d == 0.0) return OR_ZERO_PIVOT;\n            xi = xi / d;",
     "if (have_d) {\n            if (d == 0.0) return OR_ZERO_PIVOT;\n            xi = xi / d;"),
    # column-wise substitution / transpose
    ("col_sign", "x[r] = x[r] - bv[k] * x[i];", "x[r] = x[r] + bv[k] * x[i];"),
    ("col_sweep_direction", "int i = upper ? (n - 1 - t) : t;\n        if (!unit_diag) {", "int i = t;\n        if (!unit_diag) {"),
    ("transpose_operand", "return oracle_solve_col(n, row_ptr, col_idx, vals, !upper, unit_diag, g, y);",
     "return oracle_solve_row(n, row_ptr, col_idx, vals, upper, unit_diag, g, y);"),
    ("transpose_offset", "for (int k = 0; k < nnz; k++) rowT[col_idx[k] + 1] += 1;",
     "for (int k = 0; k < nnz; k++) rowT[col_idx[k]] += 1;"),
    # multi-RHS
    ("multi_wrong_ld", "F + (size_t)r * ld, X + (size_t)r * ld);", "F, X + (size_t)r * ld);"),
    # adjoint
    ("grad_transposed", "else grad_vals[k] = -grad_f[i] * x[j];", "else grad_vals[k] = -grad_f[j] * x[i];"),
    ("grad_sign", "else grad_vals[k] = -grad_f[i] * x[j];", "else grad_vals[k] = grad_f[i] * x[j];"),
    ("grad_unit_diag_kept", "if (unit_diag && j == i) grad_vals[k] = 0.0;", "if (0) grad_vals[k] = 0.0;"),
    # validation
    ("validate_no_triangle_check", "if (!upper && j > i) return OR_NOT_TRIANGULAR;", ""),
    ("validate_no_dup_check", "if (col_idx[k] == col_idx[m]) return OR_DUPLICATE;", ""),
    ("validate_no_zero_pivot", "if (vals != NULL && vals[found] == 0.0) return OR_ZERO_PIVOT;", ""),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor must be unique: %s" % name
    mut = tmp_path / ("oracle_%s.c" % name)
    mut.write_text(src.replace(old, new))
    lib_path = oracle.compile_oracle(str(mut), str(tmp_path / ("lib_%s.so" % name)))
    o = oracle.Oracle(oracle.load_library(lib_path))
    failed = []
    for pin in ALL_PINS:
        try:
            pin(o)
        except (AssertionError, ValueError, IndexError) as e:   # a caught mistake
            failed.append(pin.__name__)
    assert failed, "no pin caught mutant %s" % name
