"""FP64 eigSVDs (Alg. 3): the truncated SVD from the k largest eigenpairs of B = A^T A.

B is formed explicitly (dense, from the sparse product), its eigendecomposition is
LAPACK's symmetric solver (the library primitive standing in for eigs(B, k)), S holds the
square roots of the k largest eigenvalues (largest first), V their eigenvectors and
U = A V diag(1/S) (Alg. 3 steps 3-5). The paper states Alg. 3 for m >= n; for m < n the same
steps on A^T (B = A A^T, the smaller Gram matrix) give U and V exchanged.

Readings shared with the GPU path: eigenvalues are clamped at 0 before the square root;
singular values <= rank_tol * max are reported as 0 with zero U and V columns; the output
sign convention is that of frpca.sign_convention.

This is test infrastructure: only tests, the smoke check and the benchmark's CPU baseline
may use it.
"""
from __future__ import annotations

import numpy as np

from .frpca import sign_convention
from .sparse import csr_matmul, csr_tmatmul


def eigsvds(A, k: int, rank_tol: float = 1e-5, sign_fix: bool = True):
    """Rank-k truncated SVD of sparse A by Alg. 3. Returns (U m x k, S k descending, V n x k)."""
    if k < 1 or k > min(A.m, A.n):
        raise ValueError(f"need 1 <= k <= min(m, n); got k={k} m={A.m} n={A.n}")
    sp = A.to_scipy(np.float64)
    tall = A.m >= A.n
    B = (sp.T @ sp).toarray() if tall else (sp @ sp.T).toarray()   # step 1 (the smaller Gram)
    d, W = np.linalg.eigh(B)                                         # step 2, ascending
    top = np.arange(B.shape[0] - 1, B.shape[0] - 1 - k, -1)
    S = np.sqrt(np.maximum(d[top], 0.0))                             # step 3
    R = W[:, top]
    keep = S > rank_tol * S.max() if S.max() > 0 else np.zeros(k, bool)
    inv = np.where(keep, 1.0 / np.where(keep, S, 1.0), 0.0)          # step 4
    P = (csr_matmul(A, R) if tall else csr_tmatmul(A, R)) * inv       # step 5: A V diag(1/S)
    S = np.where(keep, S, 0.0)
    R = R * keep
    U, V = (P, R) if tall else (R, P)
    if sign_fix:
        U, V = sign_convention(U, V)
    return U, S, V
