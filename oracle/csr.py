"""CSR products and the CSR transpose, written from their definitions.

Test infrastructure (see the package docstring).  Section III-D states
that with s non-zeros the method costs O(s d); the paper does not fix a
sparse format.  Reading used here: compressed sparse row (CSR) with int32
row pointers and column indices, no duplicate (row, column) pairs.

Pinned by: tests/test_oracle_csr.py (products against the dense product of
the densified matrix; the transpose against the densified transpose, and
its entry order against the (column, row) ordering it is defined by).
"""

import numpy as np


def csr_rows(rowptr):
    """Row index of every stored entry."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    return np.repeat(np.arange(len(rowptr) - 1, dtype=np.int64), np.diff(rowptr))


def csr_matmul(rowptr, colidx, vals, m, n, X, block_rows=2000):
    """Y = A X for CSR A (m x n) and dense X (n x d), in float64.

    Row i of Y is the sum, over the stored entries (i, j, a) of row i, of
    a * X[j].  Computed in row blocks; each block forms the products of its
    entries and sums them per row (np.add.reduceat over the row starts).
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    d = X.shape[1]
    Y = np.zeros((m, d))
    for r0 in range(0, m, block_rows):
        r1 = min(m, r0 + block_rows)
        e0, e1 = rowptr[r0], rowptr[r1]
        if e1 == e0:
            continue
        counts = np.diff(rowptr[r0:r1 + 1])
        nonempty = np.nonzero(counts)[0]
        starts = rowptr[r0 + nonempty] - e0
        contrib = vals[e0:e1, None] * X[colidx[e0:e1]]
        Y[r0 + nonempty] = np.add.reduceat(contrib, starts, axis=0)
    return Y


def csr_transpose(rowptr, colidx, vals, m, n):
    """CSR of A^T (n x m).  Entries of each row of A^T (a column of A) are
    ordered by increasing row index of A, i.e. the stored entries sorted by
    (column, row).  Returns (rowptr_t int32, colidx_t int32, vals_t)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    vals = np.asarray(vals)
    rows = csr_rows(rowptr)
    # Entries are already in row order; a stable sort by column keeps it.
    order = np.argsort(colidx, kind="stable")
    counts = np.bincount(colidx, minlength=n)
    rowptr_t = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr_t[1:])
    return rowptr_t.astype(np.int32), rows[order].astype(np.int32), vals[order].copy()


def csr_to_dense(rowptr, colidx, vals, m, n):
    """Densify (float64); for small test matrices and row blocks only."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    A = np.zeros((m, n))
    rows = csr_rows(rowptr)
    A[rows, np.asarray(colidx, dtype=np.int64)] = np.asarray(vals, dtype=np.float64)
    return A
