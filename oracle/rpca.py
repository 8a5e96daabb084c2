"""FP64 basic randomized PCA: Alg. 1 (basic rPCA) and Alg. 4 (basic rPCAt) of Sections 2.2 and 3.2.

Both build an l = k + s column orthonormal basis of a sketch of A with a QR-based
orthonormalisation after every product with A or A^T, then take the SVD of the projection
of A on that basis:

* Alg. 1 sketches from the right: the basis lives on the row side of A (m x l), starting
  from orth(A Omega) with Omega an n x l Gaussian matrix; each of the p power steps
  orthonormalises A^T Q and then A G; the projection B = Q^T A is l x n, and
  U = Q U_B, V = V_B from the economic SVD B = U_B S V_B^T.
* Alg. 4 sketches from the left: the basis lives on the column side (n x l), starting from
  orth((Omega A)^T) with Omega an l x m Gaussian matrix; each power step orthonormalises
  A Q and then A^T G; the projection B = (A Q)^T is l x m, and V = Q U_B, U = V_B.

Each uses 2p + 2 passes over A. By Lemma 2 any orthonormal basis of the same range gives the
same result; here orth is LAPACK's Householder QR (numpy.linalg.qr), as in the paper's
qr(X, 0), and the SVD is LAPACK's (numpy.linalg.svd).

Readings shared with the fast algorithms and the GPU path: the Gaussian draws are Philox
normals (philox.py); the l x m draw of Alg. 4 is stored tall (m x l, element [r, j] =
normal(r*l + j)), the same long-side draw that Alg. 6 uses for even q, so that Theorem 2
holds draw for draw; singular values <= rank_tol * max are reported as exactly 0 with zero
U and V columns; the output sign convention is that of frpca.sign_convention.

This is test infrastructure: only tests, the smoke check and the benchmark's CPU baseline
may use it.
"""
from __future__ import annotations

import numpy as np

from .frpca import sign_convention
from .philox import gaussian
from .sparse import csr_matmul, csr_tmatmul


def _orth(X: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(X) by Householder QR: the Q of qr(X, 0)."""
    return np.linalg.qr(X, mode="reduced")[0]


def rpca(A, k: int, p: int, s: int, seed: int, alg: int, rank_tol: float = 1e-5, sign_fix: bool = True):
    """Rank-k truncated SVD of sparse A by the basic randomized algorithm with p power steps.

    alg = 1: Alg. 1 (basis of the row side, Omega n x l); alg = 4: Alg. 4 (basis of the
    column side, Omega l x m). Returns (U m x k, S k descending, V n x k)."""
    l = k + s
    if k < 1 or s < 0 or l > min(A.m, A.n) or p < 0 or alg not in (1, 4):
        raise ValueError(f"need 1 <= k, 0 <= s, k+s <= min(m,n), p >= 0, alg in (1, 4); "
                         f"got k={k} s={s} p={p} alg={alg} m={A.m} n={A.n}")
    mul = lambda X: csr_matmul(A, X)      # noqa: E731  X (n x l) -> A X (m x l)
    tmul = lambda Y: csr_tmatmul(A, Y)    # noqa: E731  Y (m x l) -> A^T Y (n x l)
    if alg == 1:
        Q = _orth(mul(gaussian(seed, A.n, l)))
        for _ in range(p):
            G = _orth(tmul(Q))
            Q = _orth(mul(G))
        Bt = tmul(Q)                       # B^T = A^T Q, n x l
        Vb, S, Ubt = np.linalg.svd(Bt, full_matrices=False)   # B^T = Vb S Ub^T
        U = Q @ Ubt.T[:, :k]
        V = Vb[:, :k]
    else:
        Q = _orth(tmul(gaussian(seed, A.m, l)))   # (Omega A)^T = A^T Omega^T
        for _ in range(p):
            G = _orth(mul(Q))
            Q = _orth(tmul(G))
        Bt = mul(Q)                        # B^T = A Q, m x l
        Vh, S, Uht = np.linalg.svd(Bt, full_matrices=False)   # B = Uh S Vh^T
        V = Q @ Uht.T[:, :k]
        U = Vh[:, :k]
    S = S[:k].copy()
    zero = S <= rank_tol * S.max() if S.size and S.max() > 0 else np.ones(k, bool)
    S[zero] = 0.0
    U = np.array(U)
    V = np.array(V)
    U[:, zero] = 0.0
    V[:, zero] = 0.0
    if sign_fix:
        U, V = sign_convention(U, V)
    return U, S, V
