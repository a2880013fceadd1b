"""Planted mistakes in the oracle must be caught by its pins.

Each case copies oracle/sptrsv_oracle.c, replaces one fragment with a
plausible mistake (a dropped term, a wrong sign or index, a transposed
operand, a reversed sweep), compiles the copy on the CPU and runs every pin
against it: at least one pin has to fail.  The real oracle is never touched.

A mutant can index out of bounds and corrupt the memory of the process that
runs it, so each mutant runs its pins in a child process of its own; a child
that dies before reporting (a crash) has been caught as well.
"""
import concurrent.futures as cf
import json
import os
import subprocess
import sys
import tempfile

import pytest

import oracle

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


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.dirname(os.path.abspath(__file__))

# run in a child: load the mutant library, run every pin, report the failures
_CHILD = r"""
import json, sys
sys.path[:0] = [sys.argv[2], sys.argv[3]]
import oracle
from pins import ALL_PINS
o = oracle.Oracle(oracle.load_library(sys.argv[1]))
failed = []
for pin in ALL_PINS:
    try:
        pin(o)
    except (AssertionError, ValueError, IndexError):
        failed.append(pin.__name__)
print("PINS_FAILED " + json.dumps(failed), flush=True)
"""


def _run_mutant(workdir, name, old, new):
    """(failed pin names or None if the child died first, child exit code)."""
    src = open(SRC).read()
    if src.count(old) != 1:
        return "anchor", None
    mut = os.path.join(workdir, "oracle_%s.c" % name)
    with open(mut, "w") as f:
        f.write(src.replace(old, new))
    lib_path = oracle.compile_oracle(mut, os.path.join(workdir, "lib_%s.so" % name))
    r = subprocess.run([sys.executable, "-c", _CHILD, lib_path, ROOT, TESTS], capture_output=True,
                       text=True, timeout=600, cwd=ROOT)
    for line in r.stdout.splitlines():
        if line.startswith("PINS_FAILED "):
            return json.loads(line[len("PINS_FAILED "):]), r.returncode
    return None, r.returncode


@pytest.fixture(scope="module")
def mutant_results():
    with tempfile.TemporaryDirectory(prefix="oracle_mutants_") as d:
        with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
            futs = {m[0]: ex.submit(_run_mutant, d, *m) for m in MUTANTS}
            yield {k: f.result() for k, f in futs.items()}


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_mutant_is_caught(mutant_results, name):
    failed, rc = mutant_results[name]
    assert failed != "anchor", "mutation anchor must be unique: %s" % name
    assert failed or failed is None, "no pin caught mutant %s" % name
    if failed is None:   # died before reporting: the mistake is caught by the crash
        assert rc != 0, "child of mutant %s ended without a report" % name
