/*
 * sptrsv_oracle.c -- plain, slow, obviously correct CPU oracle for sparse
 * triangular solves (Li, "On Parallel Solution of Sparse Triangular Linear
 * Systems in CUDA", arXiv:1710.04985).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code, header, table or helper with the HIP
 * library, and nothing in the library may call it.
 *
 * Everything is FP64 and single-threaded; loops follow the paper's
 * definitions in the paper's order, with no blocking or reordering.
 *
 * Conventions (readings of the paper, stated once here):
 *   - A triangle T is given as CSR (row_ptr, col_idx, vals) with n rows and
 *     the diagonal stored INSIDE each row (the paper keeps D in a separate
 *     vector d, Sec. 3; here d_i is the stored entry with col == row).
 *   - upper == 0: T is lower triangular, solve by forward substitution.
 *     upper == 1: T is upper triangular, solve by backward substitution
 *     (Sec. 3.2: the outer loop is run in reverse order).
 *   - unit_diag != 0: the diagonal is taken as 1 and any stored diagonal
 *     entry is ignored (its gradient is 0); a missing diagonal is allowed.
 *   - Levels are 0-based: a row with no off-diagonal entry has level 0 and
 *     nlev = 1 + max level.  The paper's row formula (Sec. 4.1) is 1-based;
 *     its column formula starts from zero; the two differ by exactly 1.
 *   - A dependency is a stored off-diagonal entry, whatever its value
 *     (the setup works on the nonzero pattern, Sec. 4.4).
 *   - Within one level, unknowns are listed in ascending row index.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Status codes of the oracle (its own numbering; tests map them by name). */
#define OR_OK              0
#define OR_INVALID_ARG    -1
#define OR_BAD_ROWPTR     -2
#define OR_BAD_COLIDX     -3
#define OR_NOT_TRIANGULAR -4
#define OR_DUPLICATE      -5
#define OR_MISSING_DIAG   -6
#define OR_ZERO_PIVOT     -7

/* ------------------------------------------------------------------ */
/* Validation of the problem statement, Sec. 3 eq. (1): T is triangular, */
/* every diagonal entry exists and is nonzero (unless unit diagonal).   */
/* ------------------------------------------------------------------ */
int oracle_validate(int n, int nnz, const int *row_ptr, const int *col_idx,
                    const double *vals, int upper, int unit_diag)
{
    if (n < 0 || nnz < 0) return OR_INVALID_ARG;
    if (n == 0) return (nnz == 0) ? OR_OK : OR_BAD_ROWPTR;
    if (row_ptr[0] != 0 || row_ptr[n] != nnz) return OR_BAD_ROWPTR;
    for (int i = 0; i < n; i++)
        if (row_ptr[i + 1] < row_ptr[i]) return OR_BAD_ROWPTR;
    for (int k = 0; k < nnz; k++)
        if (col_idx[k] < 0 || col_idx[k] >= n) return OR_BAD_COLIDX;
    for (int i = 0; i < n; i++) {
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
            int j = col_idx[k];
            if (!upper && j > i) return OR_NOT_TRIANGULAR;
            if (upper && j < i) return OR_NOT_TRIANGULAR;
        }
    }
    /* duplicates: compare every pair in the row (rows are short) */
    for (int i = 0; i < n; i++)
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; k++)
            for (int m = k + 1; m < row_ptr[i + 1]; m++)
                if (col_idx[k] == col_idx[m]) return OR_DUPLICATE;
    if (!unit_diag) {
        for (int i = 0; i < n; i++) {
            int found = -1;
            for (int k = row_ptr[i]; k < row_ptr[i + 1]; k++)
                if (col_idx[k] == i) found = k;
            if (found < 0) return OR_MISSING_DIAG;
            if (vals != NULL && vals[found] == 0.0) return OR_ZERO_PIVOT;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Levels, row-wise formula (Sec. 4.1):                                 */
/*   lev(i) = 1 + max{ lev(j) : T_ij stored, j != i }                   */
/* computed for i ascending (lower) or descending (upper), 0-based.     */
/* Returns nlev.                                                        */
/* ------------------------------------------------------------------ */
int oracle_levels_row(int n, const int *row_ptr, const int *col_idx,
                      int upper, int *level)
{
    int nlev = 0;
    for (int t = 0; t < n; t++) {
        int i = upper ? (n - 1 - t) : t;
        int lev = 0;                 /* no dependency -> level 0 */
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
            int j = col_idx[k];
            if (j == i) continue;
            if (level[j] + 1 > lev) lev = level[j] + 1;
        }
        level[i] = lev;
        if (lev + 1 > nlev) nlev = lev + 1;
    }
    return nlev;
}

/* ------------------------------------------------------------------ */
/* Explicit transpose of a CSR matrix (pattern and values): the CSR of   */
/* T^T is the CSC of T, i.e. (ib, jb, b) of Sec. 3.                     */
/* Entries of each output row come out in ascending source-row order.   */
/* vals / valsT may be NULL for a pattern-only transpose.               */
/* ------------------------------------------------------------------ */
void oracle_transpose(int n, const int *row_ptr, const int *col_idx,
                      const double *vals, int *rowT, int *colT, double *valsT)
{
    int nnz = row_ptr[n];
    for (int j = 0; j <= n; j++) rowT[j] = 0;
    for (int k = 0; k < nnz; k++) rowT[col_idx[k] + 1] += 1;
    for (int j = 0; j < n; j++) rowT[j + 1] += rowT[j];
    int *next = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int j = 0; j < n; j++) next[j] = rowT[j];
    for (int i = 0; i < n; i++) {
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
            int j = col_idx[k];
            int dst = next[j]++;
            colT[dst] = i;
            if (vals && valsT) valsT[dst] = vals[k];
        }
    }
    free(next);
}

/* ------------------------------------------------------------------ */
/* Levels, column-wise formula (Sec. 4.1): with lev initialised to zero, */
/* for each column j in sweep order,                                    */
/*   lev(i) = max(lev(j) + 1, lev(i)) for every i with T_ij stored.     */
/* Column access is taken from an explicit transpose of the pattern.    */
/* Returns nlev.                                                        */
/* ------------------------------------------------------------------ */
int oracle_levels_col(int n, const int *row_ptr, const int *col_idx,
                      int upper, int *level)
{
    if (n == 0) return 0;
    int nnz = row_ptr[n];
    int *ib = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    int *jb = (int *)malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    oracle_transpose(n, row_ptr, col_idx, NULL, ib, jb, NULL);
    for (int i = 0; i < n; i++) level[i] = 0;
    for (int t = 0; t < n; t++) {
        int j = upper ? (n - 1 - t) : t;       /* column j */
        for (int k = ib[j]; k < ib[j + 1]; k++) {
            int i = jb[k];                      /* T_ij stored */
            if (i == j) continue;
            if (level[j] + 1 > level[i]) level[i] = level[j] + 1;
        }
    }
    int nlev = 0;
    for (int i = 0; i < n; i++)
        if (level[i] + 1 > nlev) nlev = level[i] + 1;
    free(ib);
    free(jb);
    return nlev;
}

/* ------------------------------------------------------------------ */
/* Level sets (Sec. 4.1): jlev lists the unknowns in nondecreasing      */
/* level order (ascending row within a level), ilev[m] points to the    */
/* first entry of level m in jlev, ilev[nlev] = n.                      */
/* ------------------------------------------------------------------ */
void oracle_level_sets(int n, const int *level, int nlev, int *ilev, int *jlev)
{
    for (int m = 0; m <= nlev; m++) ilev[m] = 0;
    for (int i = 0; i < n; i++) ilev[level[i] + 1] += 1;
    for (int m = 0; m < nlev; m++) ilev[m + 1] += ilev[m];
    int *next = (int *)malloc(sizeof(int) * (size_t)(nlev > 0 ? nlev : 1));
    for (int m = 0; m < nlev; m++) next[m] = ilev[m];
    for (int i = 0; i < n; i++) jlev[next[level[i]]++] = i;
    free(next);
}

/* Dependency counts (Sec. 4.4): number of stored off-diagonal entries  */
/* in each row.                                                         */
void oracle_depcnt(int n, const int *row_ptr, const int *col_idx, int *depcnt)
{
    for (int i = 0; i < n; i++) {
        int c = 0;
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; k++)
            if (col_idx[k] != i) c++;
        depcnt[i] = c;
    }
}

/* ------------------------------------------------------------------ */
/* Row-wise substitution (Sec. 3.1; backward: Sec. 3.2).                */
/*   x(i) := f(i); x(i) -= T_ij x(j) for each stored off-diagonal j in  */
/*   stored order; x(i) := x(i) / d(i).                                 */
/* ------------------------------------------------------------------ */
int oracle_solve_row(int n, const int *row_ptr, const int *col_idx,
                     const double *vals, int upper, int unit_diag,
                     const double *f, double *x)
{
    for (int t = 0; t < n; t++) {
        int i = upper ? (n - 1 - t) : t;
        double xi = f[i];
        double d = 1.0;
        int have_d = 0;
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
            int j = col_idx[k];
            if (j == i) { d = vals[k]; have_d = 1; continue; }
            xi = xi - vals[k] * x[j];
        }
        if (!unit_diag) {
            if (!have_d || d == 0.0) return OR_ZERO_PIVOT;
            xi = xi / d;
        }
        x[i] = xi;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Column-wise substitution on a CSC matrix (Sec. 3.2):                 */
/*   x := f; for each column i in sweep order: x(i) := x(i)/d(i); then  */
/*   x(jb(k)) -= b(k) x(i) for every stored off-diagonal entry of col i. */
/* (ib, jb, bv) is the CSC of the triangle; upper selects the sweep.    */
/* ------------------------------------------------------------------ */
int oracle_solve_col(int n, const int *ib, const int *jb, const double *bv,
                     int upper, int unit_diag, const double *f, double *x)
{
    for (int i = 0; i < n; i++) x[i] = f[i];
    for (int t = 0; t < n; t++) {
        int i = upper ? (n - 1 - t) : t;
        if (!unit_diag) {
            double d = 0.0;
            int have_d = 0;
            for (int k = ib[i]; k < ib[i + 1]; k++)
                if (jb[k] == i) { d = bv[k]; have_d = 1; }
            if (!have_d || d == 0.0) return OR_ZERO_PIVOT;
            x[i] = x[i] / d;
        }
        for (int k = ib[i]; k < ib[i + 1]; k++) {
            int r = jb[k];
            if (r == i) continue;
            x[r] = x[r] - bv[k] * x[i];
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Transposed solve T^T y = g, reading the CSR of T as the CSC of T^T   */
/* and running the column-wise sweep of Sec. 3.2 on it.  T^T of a lower */
/* triangle is upper, so the sweep runs backward, and vice versa.       */
/* ------------------------------------------------------------------ */
int oracle_solve_transpose(int n, const int *row_ptr, const int *col_idx,
                           const double *vals, int upper, int unit_diag,
                           const double *g, double *y)
{
    /* column i of T^T == row i of T */
    return oracle_solve_col(n, row_ptr, col_idx, vals, !upper, unit_diag, g, y);
}

/* Several right-hand sides, column-major with leading dimension ld:    */
/* one row-wise substitution per column.                                */
int oracle_solve_multi(int n, const int *row_ptr, const int *col_idx,
                       const double *vals, int upper, int unit_diag,
                       int nrhs, int ld, const double *F, double *X)
{
    for (int r = 0; r < nrhs; r++) {
        int st = oracle_solve_row(n, row_ptr, col_idx, vals, upper, unit_diag,
                                  F + (size_t)r * ld, X + (size_t)r * ld);
        if (st != OR_OK) return st;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Adjoint of x = T^{-1} f with respect to the stored values of T:      */
/* with grad_f = T^{-T} grad_x, d(loss)/d T_ij = -grad_f(i) * x(j) for  */
/* every stored entry (i, j); 0 for a stored diagonal under unit_diag.  */
/* ------------------------------------------------------------------ */
void oracle_grad_vals(int n, const int *row_ptr, const int *col_idx,
                      int unit_diag, const double *grad_f, const double *x,
                      double *grad_vals)
{
    for (int i = 0; i < n; i++) {
        for (int k = row_ptr[i]; k < row_ptr[i + 1]; k++) {
            int j = col_idx[k];
            if (unit_diag && j == i) grad_vals[k] = 0.0;
            else grad_vals[k] = -grad_f[i] * x[j];
        }
    }
}
