"""Sparse test matrices (seeded, synthetic).

The paper's sparse experiments (Section 8) run on matrices from a public
collection, which is not available here.  The stand-in is an m x n matrix with
exactly ``per_row`` stored entries in every row, at distinct columns drawn
uniformly at random, values N(0, 1) times row_scale(i) (by default i^-1/2 for
the 1-indexed row i), column indices sorted within each row.  Both CSR and CSC
(the CSR of A^T) are returned, as NumPy int32 / float32 arrays.
"""

import numpy as np


def random_rows(m, n, per_row, seed, decay=0.5):
    """CSR (row_ptr, col_idx, val) of the matrix described above."""
    if per_row > n:
        raise ValueError("per_row must not exceed n")
    rng = np.random.default_rng(seed)
    cols = rng.integers(0, n, size=(m, per_row), dtype=np.int64)
    cols.sort(axis=1)
    # redraw the rows that hold a repeated column until every row is distinct
    while True:
        bad = np.flatnonzero(np.any(cols[:, 1:] == cols[:, :-1], axis=1))
        if bad.size == 0:
            break
        redraw = rng.integers(0, n, size=(bad.size, per_row), dtype=np.int64)
        redraw.sort(axis=1)
        cols[bad] = redraw
    scale = np.arange(1, m + 1, dtype=np.float64) ** (-decay)
    val = (rng.standard_normal((m, per_row)) * scale[:, None]).astype(np.float32)
    row_ptr = (np.arange(m + 1, dtype=np.int64) * per_row).astype(np.int32)
    return row_ptr, cols.reshape(-1).astype(np.int32), val.reshape(-1)


def transpose(m, n, row_ptr, col_idx, val):
    """CSC of the same matrix (col_ptr, row_idx, val_t): rows of A^T, row
    indices ascending within each column."""
    col_idx = np.asarray(col_idx, dtype=np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    order = np.lexsort((rows, col_idx))
    counts = np.bincount(col_idx, minlength=n)
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=col_ptr[1:])
    return (col_ptr.astype(np.int32), rows[order].astype(np.int32),
            np.asarray(val, dtype=np.float32)[order])


def to_scipy(m, n, row_ptr, col_idx, val):
    import scipy.sparse as sp
    return sp.csr_matrix((np.asarray(val), np.asarray(col_idx), np.asarray(row_ptr)), shape=(m, n))
