"""Pins of the oracle's centred mode: principal components of A - 1 mu^T (mu = column means
of A), which the paper's PCA assumes (data centred before the SVD, Section 1) and which the
method reaches without forming the dense matrix.

Each check compares with something other than the centred code itself: the explicitly
centred dense matrix (its products, and its exact SVD by a from-scratch Jacobi SVD when the
subspace is full), the zero column means of the component scores, and finite differences of
a loss evaluated with LAPACK's SVD of the centred dense matrix rebuilt from perturbed values.
A centring term left out of the adjoint fails the finite-difference check.
"""
import numpy as np
import pytest

import oracle
from refs import jacobi_svd
from synth import random_sparse, small_decay


def _dense_centred(A):
    D = A.toarray().astype(np.float64)
    return D - D.mean(axis=0)


def test_centred_products_match_dense():
    A = random_sparse(40, 25, 0.3, seed=51)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((25, 7))
    Y = rng.standard_normal((40, 7))
    Dc = _dense_centred(A)
    mul, tmul = oracle.products(A, center=True)
    np.testing.assert_allclose(mul(X), Dc @ X, atol=1e-12)
    np.testing.assert_allclose(tmul(Y), Dc.T @ Y, atol=1e-12)
    mul0, tmul0 = oracle.products(A)
    np.testing.assert_allclose(mul0(X), A.toarray() @ X, atol=1e-12)
    np.testing.assert_allclose(tmul0(Y), A.toarray().T @ Y, atol=1e-12)


@pytest.mark.parametrize("q", [2, 3, 4])
@pytest.mark.parametrize("shape", [(16, 10), (10, 16)])
def test_centred_full_subspace_is_exact_svd_of_centred_matrix(q, shape):
    # l = min(m, n): the sketch spans everything, so the result is the SVD of A - 1 mu^T
    A = random_sparse(*shape, 0.5, seed=52)
    l = min(shape)
    k, s = l - 3, 3
    U, S, V, _ = oracle.frpca(A, k, q, s, seed=5, center=True)
    Uj, Sj, Vj = jacobi_svd(_dense_centred(A))
    np.testing.assert_allclose(S, Sj[:k], rtol=1e-10)
    for i in range(k):
        assert abs(abs(U[:, i] @ Uj[:, i]) - 1) < 1e-9
        assert abs(abs(V[:, i] @ Vj[:, i]) - 1) < 1e-9
    # and differs from the SVD of A itself
    Sa = np.linalg.svd(A.toarray(), compute_uv=False)
    assert np.abs(S[0] - Sa[0]) > 1e-3 * Sa[0]


def test_centred_scores_have_zero_mean():
    # U = (A - 1 mu^T) V S^-1, and 1^T (A - 1 mu^T) = 0
    A = small_decay()
    U, S, V, _ = oracle.frpca(A, 10, 3, 5, seed=20181015, center=True)
    assert np.abs(U.sum(axis=0)).max() < 1e-10
    U0, *_ = oracle.frpca(A, 10, 3, 5, seed=20181015)
    assert np.abs(U0.sum(axis=0)).max() > 1e-3


def _loss_terms(k, m, n, seed):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((m, k))
    Dd = rng.standard_normal((n, k))
    w = rng.random(k) + 0.5
    w2 = rng.random(k) + 0.5

    def loss(U, S, V):
        return S.sum() + (w * ((C * U).sum(0)) ** 2).sum() + (w2 * ((Dd * V).sum(0)) ** 2).sum()

    def grads(U, S, V):
        return (2 * C * (w * (C * U).sum(0))[None, :], np.ones(k), 2 * Dd * (w2 * (Dd * V).sum(0))[None, :])

    return loss, grads


def _topk_centred(D, k):
    U, S, Vt = np.linalg.svd(D - D.mean(axis=0), full_matrices=False)
    return U[:, :k], S[:k], Vt[:k].T


@pytest.mark.parametrize("center_in_adjoint", [True, False])
def test_centred_adjoint_matches_fd(center_in_adjoint):
    # D = 1 b^T + (centred rank-k part): A - 1 mu^T has exact rank k with distinct singular
    # values, where every term of the adjoint is exact. All entries are stored.
    m, n, k = 24, 15, 4
    rng = np.random.default_rng(61)
    Z = rng.standard_normal((m, k)) @ np.diag(np.linspace(3.0, 1.0, k)) @ rng.standard_normal((k, n))
    Z -= Z.mean(axis=0)
    D = Z + np.outer(np.ones(m), rng.standard_normal(n))
    rows, cols = np.nonzero(np.ones((m, n)))
    loss, grads = _loss_terms(k, m, n, seed=62)
    U, S, V = _topk_centred(D, k)
    g = oracle.svd_adjoint_values(U, S, V, *grads(U, S, V), rows, cols, center=center_in_adjoint)
    idx = range(0, rows.size, 5)
    fd = np.empty(len(idx))
    for t, e in enumerate(idx):
        r, c = rows[e], cols[e]
        h = 1e-6 * max(abs(D[r, c]), 0.05)
        Dp = D.copy()
        Dp[r, c] += h
        Dm = D.copy()
        Dm[r, c] -= h
        fd[t] = (loss(*_topk_centred(Dp, k)) - loss(*_topk_centred(Dm, k))) / (2 * h)
    err = np.abs(g[list(idx)] - fd).max() / np.abs(fd).max()
    if center_in_adjoint:
        assert err < 1e-5
    else:  # the adjoint of the uncentred map misses the column-mean term
        assert err > 1e-3
