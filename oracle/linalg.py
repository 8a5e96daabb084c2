"""Dense FP64 building blocks of the method: LU basis (Lemma 3) and eigSVD (Alg. 2).

This is test infrastructure: only tests, the smoke check and the benchmark's CPU baseline
may use it.
"""
from __future__ import annotations

import numpy as np


def lu_pl(X: np.ndarray, tol: float = 1e-12):
    """The first output of [Q, ~] = lu(X): the n x l factor P^T L of P X = L U (eq. 8).

    Gaussian elimination with partial pivoting on the columns of X in order (Section 3.1,
    Lemma 3): at step j the pivot is the not-yet-used row with the largest |entry| in
    column j (ties go to the lowest row index), column j of L is that column divided by
    the pivot (zero on rows already used as pivots, one on the pivot row), and the pivot
    row's multiple is subtracted from the remaining rows. The rows are left in their
    original order, which is P^T L.

    Rank guard (the paper assumes full rank; this is the reading used for exact-recovery
    inputs): if the largest remaining |entry| of column j is <= tol * max|X|, the column is
    numerically dependent on the earlier ones; column j of L is set to zero and no pivot
    row is consumed.

    Returns (Q, pivots, dropped) with pivots the row index used at each kept step and
    dropped the list of zeroed columns.
    """
    A = np.array(X, dtype=np.float64, copy=True)
    n, l = A.shape
    scale = float(np.abs(A).max()) if A.size else 0.0
    L = np.zeros((n, l))
    free = np.ones(n, dtype=bool)
    pivots, dropped = [], []
    for j in range(l):
        cand = np.where(free, np.abs(A[:, j]), -1.0)
        p = int(np.argmax(cand))
        if not free[p] or cand[p] <= tol * scale or scale == 0.0:
            dropped.append(j)
            continue
        piv = A[p, j]
        lj = np.where(free, A[:, j] / piv, 0.0)
        lj[p] = 1.0
        L[:, j] = lj
        free[p] = False
        upd = lj.copy()
        upd[~free] = 0.0  # rows already used as pivots (including p) keep their values
        A[:, j + 1:] -= np.outer(upd, A[p, j + 1:])
        pivots.append(p)
    return L, pivots, dropped


def eig_asc(B: np.ndarray):
    """Eigendecomposition of a symmetric matrix, eigenvalues ascending (Alg. 2 step 2).

    LAPACK's symmetric eigensolver (through numpy) serves as the library primitive; the
    paper notes that eig returns ascending order, which the final steps of Alg. 5/6 rely on.
    """
    d, V = np.linalg.eigh(np.asarray(B, dtype=np.float64))
    return d, V


def eigsvd(X: np.ndarray, tol: float = 1e-12):
    """eigSVD (Alg. 2): economic SVD of a tall X through the eigendecomposition of X^T X.

    B = X^T X; [V, D] = eig(B); S = sqrt(diag(D)); U = X V diag(1/S). Singular values come
    out ascending (Section 3.1). Readings for rank-deficient X, which the paper excludes:
    eigenvalues are clamped at zero before the square root, and values S_j <= tol * max(S)
    are treated as zero, with 1/S_j replaced by 0 so that column j of U is zero.

    Returns (U, S, V, ndropped).
    """
    X = np.asarray(X, dtype=np.float64)
    B = X.T @ X
    d, V = eig_asc(B)
    S = np.sqrt(np.maximum(d, 0.0))
    smax = float(S.max()) if S.size else 0.0
    keep = S > tol * smax
    sinv = np.zeros_like(S)
    np.divide(1.0, S, out=sinv, where=keep)
    U = (X @ V) * sinv[None, :]
    S = np.where(keep, S, 0.0)
    return U, S, V, int((~keep).sum())
