"""FP64 frPCA (Alg. 5, m <= n) and frPCAt (Alg. 6, m >= n) of Section 3.3.

What the method computes, for a sketch width l = k + s and q passes over A (q >= 2):

* a starting basis of l columns on the short side of A: for odd q the Gaussian matrix
  itself (the modified power iteration of Section 3.2, which saves one pass), for even q
  the product of A with a Gaussian matrix drawn on the long side, reduced to a basis;
* floor((q - 1) / 2) power steps, each applying A and A^T once and replacing the basis by
  a basis of the result: the LU factor P^T L of Lemma 3 (eq. 8) in every step but the
  last, eigSVD (Alg. 2) in the last one (and after the start when q = 2, where there is
  no power step);
* a Rayleigh-Ritz step: eigSVD of A applied to the final basis gives l singular triplets
  in ascending order, of which the k largest are kept, largest first.

Alg. 5 and Alg. 6 are the same computation with A and A^T exchanged (U and V swap
roles), so one routine runs both on an operator whose rows are the long side.

Readings where the paper is silent (each also applied by the GPU path):
  * centring (option): the PCA of data with rows as samples centres the columns; the
    products then act on A - 1 mu^T without forming it (see products());
  * orientation: m >= n runs Alg. 6, m < n runs Alg. 5 (the paper picks by shape and uses
    Alg. 6 on a square matrix in Section 4.2);
  * the Gaussian draws come from Philox4x32-10 (see philox.py); the long-side draw of even
    q is stored tall (rows of the long side, l columns), element [r, j] = normal(r*l + j),
    which is the transpose of the paper's l x (long side) matrix;
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


def pass_schedule(q: int):
    """How q passes are spent (Section 3.3): returns (start, bases) where start is "gaussian"
    (odd q: the Gaussian matrix is the first basis, no pass) or "sketch" (even q: one pass
    with a long-side Gaussian matrix, followed by a basis), and bases lists the basis taken
    after the start sketch (even q only) and after each power step, in order: "lu" or "eig".
    Every power step costs two passes and the Rayleigh-Ritz step one."""
    steps = (q - 1) // 2
    if q % 2 == 0:
        start = "sketch"
        bases = ["eig" if steps == 0 else "lu"]
    else:
        start = "gaussian"
        bases = []
    bases += ["lu"] * max(steps - 1, 0) + (["eig"] if steps else [])
    return start, bases


def _basis(X: np.ndarray, kind: str, inner_tol: float) -> np.ndarray:
    """A basis of range(X): the LU factor P^T L (Lemma 3) or the eigSVD left factor (Alg. 2)."""
    return lu_pl(X, inner_tol)[0] if kind == "lu" else eigsvd(X, inner_tol)[0]


def randomized_svd(fwd, back, long_rows: int, short_rows: int, k: int, q: int, s: int, seed: int,
                   rank_tol: float = 1e-5, inner_tol: float = 1e-12, log=None):
    """Rank-k SVD of an operator M (long_rows x short_rows, long_rows >= short_rows) given by
    fwd: X -> M X and back: Y -> M^T Y, by the pass schedule of Section 3.3.

    Returns (P long_rows x k, S k descending, R short_rows x k) with M ~ P diag(S) R^T.
    log (optional) receives a line after each pass."""
    say = log or (lambda msg: None)
    l = k + s
    start, bases = pass_schedule(q)
    todo = iter(bases)
    if start == "sketch":
        Q = _basis(back(gaussian(seed, long_rows, l)), next(todo), inner_tol)
        say("start: sketch of the long-side Gaussian matrix and its basis")
    else:
        Q = gaussian(seed, short_rows, l)
        say("start: short-side Gaussian matrix")
    for step, kind in enumerate(todo, 1):
        Q = _basis(back(fwd(Q)), kind, inner_tol)
        say(f"power step {step}: {kind} basis")
    # Rayleigh-Ritz: eigSVD of M Q; eigSVD lists singular values ascending, so the k largest
    # are its last k columns, taken largest first
    W, sig, Z, _ = eigsvd(fwd(Q), rank_tol)
    top = np.arange(l - 1, l - 1 - k, -1)
    say("final eigSVD")
    return W[:, top], sig[top], Q @ Z[:, top]


def frpca(A, k: int, q: int, s: int, seed: int, rank_tol: float = 1e-5, inner_tol: float = 1e-12,
          sign_fix: bool = True, center: bool = False, log=None):
    """Rank-k truncated SVD of sparse A (or, with center, of A - 1 mu^T) by frPCA / frPCAt
    with q passes and oversampling s.

    Returns (U, S, V, info) with info = {"orientation": "alg6"|"alg5", "rank_dropped": r}.
    """
    check_args(A.m, A.n, k, q, s)
    mul, tmul = products(A, center)
    if A.m >= A.n:
        # Alg. 6: the operator is A, its rows (the long side) carry U
        U, S, V = randomized_svd(mul, tmul, A.m, A.n, k, q, s, seed, rank_tol, inner_tol, log)
        orient = "alg6"
    else:
        # Alg. 5: the same schedule on A^T, whose rows carry V
        V, S, U = randomized_svd(tmul, mul, A.n, A.m, k, q, s, seed, rank_tol, inner_tol, log)
        orient = "alg5"
    zero = S == 0.0
    U[:, zero] = 0.0
    V[:, zero] = 0.0
    if sign_fix:
        U, V = sign_convention(U, V)
    return U, S, V, {"orientation": orient, "rank_dropped": int(zero.sum())}
