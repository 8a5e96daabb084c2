"""FP64 frPCA (Alg. 5, m <= n) and frPCAt (Alg. 6, m >= n), step by step.

The two algorithms are written out separately, each following its own listing in the
paper's order and notation (Section 3.3). The pass parameter q (the number of passes over
A, q >= 2) selects the start: for even q the sketch is one product with a Gaussian matrix
followed by LU (q > 2) or eigSVD (q = 2); for odd q the Gaussian matrix itself is the
starting basis (the modified power iteration of Section 3.2). floor((q-1)/2) power steps
follow, each a product with A and A^T and an LU basis, the last one an eigSVD basis; a final
eigSVD of the projected matrix gives the k leading triplets, taken in the order
ind = k+s, k+s-1, ..., s+1 because eigSVD returns ascending singular values.

Readings where the paper is silent (each also applied by the GPU path):
  * centring (option): the PCA of data with rows as samples centres the columns; the
    products then act on A - 1 mu^T without forming it (see products());
  * orientation: m >= n runs Alg. 6, m < n runs Alg. 5 (the paper picks by shape and uses
    Alg. 6 on a square matrix in Section 4.2);
  * the Gaussian draws come from Philox4x32-10 (see philox.py); Alg. 6's randn(k+s, m)
    is drawn as its m x (k+s) transpose, element [r, j] = normal(r*(k+s) + j);
  * rank guards (see linalg.py). Inner LU and eigSVD bases only guard against division by
    a numerically zero pivot or singular value (inner_tol, relative); the final eigSVD
    reports singular values <= rank_tol * max as exactly zero, with zero U and V columns.
    eigSVD squares the condition number, so it cannot resolve singular values below about
    sqrt(unit roundoff) * sigma_max; rank_tol = 1e-5 sits above that floor for FP64 and for
    a Gram matrix of FP32 data, and both the oracle and the GPU path use it;
  * output sign: each pair (u_i, v_i) is flipped so that the largest-magnitude entry of
    v_i is positive (ties: lowest index). The paper leaves signs free.

This is test infrastructure: only tests, the smoke check and the benchmark's CPU baseline
may use it.
"""
from __future__ import annotations

import numpy as np

from .linalg import eigsvd, lu_pl
from .philox import gaussian
from .sparse import csr_matmul, csr_tmatmul


def check_args(m: int, n: int, k: int, q: int, s: int) -> None:
    """Argument rules shared with the C interface: 1 <= k, 0 <= s, k+s <= min(m, n), q >= 2."""
    if k < 1 or s < 0 or k + s > min(m, n):
        raise ValueError(f"need 1 <= k, 0 <= s, k+s <= min(m,n); got k={k} s={s} m={m} n={n}")
    if q < 2:
        raise ValueError(f"the pass parameter q must be >= 2 (Alg. 5/6); got {q}")


def sign_convention(U: np.ndarray, V: np.ndarray):
    """Flip (u_i, v_i) jointly so that the largest-|.| entry of v_i is positive."""
    U = U.copy()
    V = V.copy()
    for i in range(V.shape[1]):
        j = int(np.argmax(np.abs(V[:, i])))
        if V[j, i] < 0:
            U[:, i] = -U[:, i]
            V[:, i] = -V[:, i]
    return U, V


def products(A, center: bool = False):
    """The two products the algorithms use, (X -> A X, Y -> A^T Y), of A itself or, with
    center, of the column-centred matrix A - 1 mu^T (mu = column means of A, the data
    centring the paper's PCA assumes in Section 1), written without forming it:
    (A - 1 mu^T) X = A X - 1 (mu^T X) and (A - 1 mu^T)^T Y = A^T Y - mu (1^T Y)."""
    if not center:
        return (lambda X: csr_matmul(A, X)), (lambda Y: csr_tmatmul(A, Y))
    mu = csr_tmatmul(A, np.ones((A.m, 1)))[:, 0] / A.m

    def mul(X):
        X = np.asarray(X, dtype=np.float64)
        return csr_matmul(A, X) - (mu @ X)[None, :]

    def tmul(Y):
        Y = np.asarray(Y, dtype=np.float64)
        return csr_tmatmul(A, Y) - np.outer(mu, Y.sum(axis=0))

    return mul, tmul


def frpcat(A, k: int, q: int, s: int, seed: int, rank_tol: float = 1e-5,
           inner_tol: float = 1e-12, center: bool = False):
    """Alg. 6 (frPCAt) for m >= n. Returns (U m x k, S k descending, V n x k)."""
    mul, tmul = products(A, center)
    l = k + s
    if q % 2 == 0:
        omega_t = gaussian(seed, A.m, l)          # randn(k+s, m), stored transposed
        Q = tmul(omega_t)                         # Q = (Omega A)^T
        if q == 2:
            Q = eigsvd(Q, inner_tol)[0]
        else:
            Q = lu_pl(Q, inner_tol)[0]
    else:
        Q = gaussian(seed, A.n, l)                # Q = randn(n, k+s)
    last = (q - 1) // 2
    for i in range(1, last + 1):
        X = tmul(mul(Q))                          # A^T (A Q)
        if i == last:
            Q = eigsvd(X, inner_tol)[0]
        else:
            Q = lu_pl(X, inner_tol)[0]
    Uh, Sh, Vh, _ = eigsvd(mul(Q), rank_tol)
    ind = np.arange(l - 1, s - 1, -1)             # k+s : -1 : s+1, zero-based
    U = Uh[:, ind]
    V = Q @ Vh[:, ind]
    S = Sh[ind]
    return U, S, V


def frpca_alg5(A, k: int, q: int, s: int, seed: int, rank_tol: float = 1e-5,
               inner_tol: float = 1e-12, center: bool = False):
    """Alg. 5 (frPCA) for m <= n. Returns (U m x k, S k descending, V n x k)."""
    mul, tmul = products(A, center)
    l = k + s
    if q % 2 == 0:
        Q = gaussian(seed, A.n, l)                # Q = randn(n, k+s)
        Q = mul(Q)                                # Q = A Q
        if q > 2:
            Q = lu_pl(Q, inner_tol)[0]
        else:
            Q = eigsvd(Q, inner_tol)[0]
    else:
        Q = gaussian(seed, A.m, l)                # Q = randn(m, k+s)
    last = (q - 1) // 2
    for i in range(1, last + 1):
        X = mul(tmul(Q))                          # A (A^T Q)
        if i == last:
            Q = eigsvd(X, inner_tol)[0]
        else:
            Q = lu_pl(X, inner_tol)[0]
    Uh, Sh, Vh, _ = eigsvd(tmul(Q), rank_tol)
    ind = np.arange(l - 1, s - 1, -1)
    U = Q @ Vh[:, ind]
    V = Uh[:, ind]
    S = Sh[ind]
    return U, S, V


def frpca(A, k: int, q: int, s: int, seed: int, rank_tol: float = 1e-5, inner_tol: float = 1e-12,
          sign_fix: bool = True, center: bool = False):
    """Rank-k truncated SVD of sparse A (or, with center, of A - 1 mu^T) by frPCA / frPCAt
    with q passes and oversampling s.

    Returns (U, S, V, info) with info = {"orientation": "alg6"|"alg5", "rank_dropped": r}.
    """
    check_args(A.m, A.n, k, q, s)
    if A.m >= A.n:
        U, S, V = frpcat(A, k, q, s, seed, rank_tol, inner_tol, center)
        orient = "alg6"
    else:
        U, S, V = frpca_alg5(A, k, q, s, seed, rank_tol, inner_tol, center)
        orient = "alg5"
    zero = S == 0.0
    U[:, zero] = 0.0
    V[:, zero] = 0.0
    if sign_fix:
        U, V = sign_convention(U, V)
    return U, S, V, {"orientation": orient, "rank_dropped": int(zero.sum())}
