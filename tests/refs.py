"""Independent references that pin the oracle (never used by the oracle or the GPU path).

* ``jacobi_svd``: one-sided (Hestenes) Jacobi SVD written from scratch for tiny dense
  matrices (Demmel & Veselic, SIAM J. Matrix Anal. Appl. 13(4), 1992).
* ``rpca_basic`` / ``rpcat_basic``: the textbook randomized SVD with QR orthonormalisation
  and a dense SVD of the projected matrix (Alg. 1 and Alg. 4); by Theorems 1 and 2 they
  equal Alg. 5 and Alg. 6 for even pass counts with p = (q-2)/2 and the same Gaussian draws.
* ``subspace_iteration``: the odd-pass variant of Section 3.2 written as plain QR subspace
  iteration started from the Gaussian matrix itself.
* metrics: largest principal angle (as its sine) and relative singular-value error.
"""
from __future__ import annotations

import numpy as np


def jacobi_svd(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Economic SVD (U, s descending, V) of a small dense matrix by one-sided Jacobi."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        V, s, U = jacobi_svd(A.T, tol, max_sweeps)
        return U, s, V
    W = A.copy()
    V = np.eye(n)
    for _ in range(max_sweeps):
        rotated = False
        for p in range(n - 1):
            for q in range(p + 1, n):
                a = W[:, p] @ W[:, p]
                b = W[:, q] @ W[:, q]
                g = W[:, p] @ W[:, q]
                if abs(g) <= tol * np.sqrt(a * b) or g == 0.0:
                    continue
                rotated = True
                zeta = (b - a) / (2.0 * g)
                t = np.sign(zeta) / (abs(zeta) + np.sqrt(1.0 + zeta * zeta)) if zeta != 0 else 1.0
                c = 1.0 / np.sqrt(1.0 + t * t)
                s_ = c * t
                wp, wq = W[:, p].copy(), W[:, q].copy()
                W[:, p], W[:, q] = c * wp - s_ * wq, s_ * wp + c * wq
                vp, vq = V[:, p].copy(), V[:, q].copy()
                V[:, p], V[:, q] = c * vp - s_ * vq, s_ * vp + c * vq
        if not rotated:
            break
    s = np.sqrt((W * W).sum(0))
    order = np.argsort(-s, kind="stable")
    s = s[order]
    W = W[:, order]
    V = V[:, order]
    U = np.zeros_like(W)
    nz = s > 0
    U[:, nz] = W[:, nz] / s[nz]
    return U, s, V


def _orth(X):
    return np.linalg.qr(X, mode="reduced")[0]


def rpca_basic(A: np.ndarray, k: int, p: int, omega: np.ndarray):
    """Alg. 1 with Omega given (n x l): QR orthonormalisation, dense SVD of B = Q^T A."""
    Q = _orth(A @ omega)
    for _ in range(p):
        G = _orth(A.T @ Q)
        Q = _orth(A @ G)
    B = Q.T @ A
    Ub, S, Vt = np.linalg.svd(B, full_matrices=False)
    return (Q @ Ub)[:, :k], S[:k], Vt.T[:, :k]


def rpcat_basic(A: np.ndarray, k: int, p: int, omega_lm: np.ndarray):
    """Alg. 4 with Omega given (l x m): left sketch, dense SVD of B = (A Q)^T."""
    Q = _orth((omega_lm @ A).T)
    for _ in range(p):
        G = _orth(A @ Q)
        Q = _orth(A.T @ G)
    B = (A @ Q).T
    Uh, S, Vht = np.linalg.svd(B, full_matrices=False)
    return Vht.T[:, :k], S[:k], (Q @ Uh)[:, :k]


def subspace_iteration(A: np.ndarray, k: int, nit: int, omega: np.ndarray, right: bool = True):
    """Odd-pass scheme: Q0 = Omega; nit x Q = qr(A^T A Q) (or A A^T Q); SVD of the projection."""
    if right:  # Omega is n x l, basis of the row space
        Q = _orth(omega)
        for _ in range(nit):
            Q = _orth(A.T @ (A @ Q))
        Ub, S, Wt = np.linalg.svd(A @ Q, full_matrices=False)
        return Ub[:, :k], S[:k], (Q @ Wt.T)[:, :k]
    Q = _orth(omega)  # m x l, basis of the column space
    for _ in range(nit):
        Q = _orth(A @ (A.T @ Q))
    Vb, S, Wt = np.linalg.svd(A.T @ Q, full_matrices=False)
    return (Q @ Wt.T)[:, :k], S[:k], Vb[:, :k]


def sin_theta(Uref: np.ndarray, U: np.ndarray) -> float:
    """Sine of the largest principal angle between range(Uref) and range(U) (both orthonormal)."""
    Uref = np.asarray(Uref, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    if U.shape[1] == 0:
        return 0.0
    R = U - Uref @ (Uref.T @ U)
    return float(np.linalg.norm(R, 2))


def sigma_rel_err(Sref, S, floor: float = 1e-6) -> float:
    Sref = np.asarray(Sref, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    keep = Sref > floor * Sref.max()
    if not keep.any():
        return 0.0
    return float(np.max(np.abs(S[keep] - Sref[keep]) / Sref[keep]))


def orth_err(U: np.ndarray) -> float:
    U = np.asarray(U, dtype=np.float64)
    return float(np.abs(U.T @ U - np.eye(U.shape[1])).max())
