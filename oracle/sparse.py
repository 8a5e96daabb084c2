"""Sparse products and the transposed (column-major) storage, in FP64, for the oracle.

The paper multiplies the CSR matrix A by tall dense matrices from both sides (A Q and
A^T Y, Alg. 5/6) and notes that forming A^T is awkward in the usual sparse storage
(Section 3.2). The oracle uses scipy's sparse product as a library matmul and defines the
transposed storage plainly: nonzeros stably sorted by column.

Matrices are any object with attributes m, n, row_ptr, col, val (CSR, canonical form).
This is test infrastructure: only tests, the smoke check and the benchmark's CPU baseline
may use it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def to_scipy(A) -> sp.csr_matrix:
    return sp.csr_matrix(
        (np.asarray(A.val, dtype=np.float64), np.asarray(A.col, dtype=np.int64),
         np.asarray(A.row_ptr, dtype=np.int64)),
        shape=(A.m, A.n),
    )


def csr_matmul(A, X: np.ndarray) -> np.ndarray:
    """A @ X in FP64 (A is m x n sparse, X is n x l dense)."""
    X = np.asarray(X, dtype=np.float64)
    assert X.shape[0] == A.n
    return np.asarray(to_scipy(A) @ X)


def csr_tmatmul(A, Y: np.ndarray) -> np.ndarray:
    """A^T @ Y in FP64 (A is m x n sparse, Y is m x l dense)."""
    Y = np.asarray(Y, dtype=np.float64)
    assert Y.shape[0] == A.m
    return np.asarray(to_scipy(A).T @ Y)


def csc_mirror(A):
    """Column-major copy of A's pattern: (col_ptr int64[n+1], row int32[nnz], perm int64[nnz]).

    perm[e'] is the CSR position of the e'-th nonzero in column-major order, obtained by a
    stable sort of the CSR positions by column, so rows ascend within each column.
    """
    col = np.asarray(A.col, dtype=np.int64)
    perm = np.argsort(col, kind="stable")
    counts = np.bincount(col, minlength=A.n)
    col_ptr = np.zeros(A.n + 1, np.int64)
    np.cumsum(counts, out=col_ptr[1:])
    rows_of = np.repeat(np.arange(A.m, dtype=np.int64), np.diff(np.asarray(A.row_ptr)))
    return col_ptr, rows_of[perm].astype(np.int32), perm


def transpose(A):
    """A^T as a CSR-shaped object (the Alg. 5 <-> Alg. 6 orientation swap in tests)."""
    col_ptr, row, perm = csc_mirror(A)

    class _T:
        pass

    t = _T()
    t.m, t.n = A.n, A.m
    t.row_ptr, t.col, t.val = col_ptr, row, np.asarray(A.val)[perm]
    return t
