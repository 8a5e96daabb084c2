"""Pins of the oracle's truncated-SVD adjoint (the differentiated form of the method).

Finite differences of losses evaluated with LAPACK's dense SVD in FP64 pin the formula:
on an exactly rank-k input every term of the adjoint is exact, so a dropped term or a wrong
sign fails; the sigma-sum gradient u_i v_i^T is exact for any k; and ||U_k W||^2 is
invariant (U_k^T U_k = I), so its gradient is exactly zero.
"""
import numpy as np
import pytest

import oracle
from synth import zipf_normal


def _exact_rank_pattern(m, n, k, seed):
    """FP64 sparse matrix of exact rank k: sum of k outer products of sparse vectors.

    The supports overlap (each factor has density 1/2), so at stored positions the
    off-diagonal coupling terms of the adjoint contribute; the singular values are distinct.
    """
    rng = np.random.default_rng(seed)
    Uf = rng.standard_normal((m, k)) * (rng.random((m, k)) < 0.5)
    Vf = rng.standard_normal((n, k)) * (rng.random((n, k)) < 0.5)
    D = Uf @ np.diag(np.linspace(3.0, 1.0, k)) @ Vf.T
    rows, cols = np.nonzero(D)
    S = np.linalg.svd(D, compute_uv=False)
    assert S[k - 1] > 1e-3 * S[0] and S[k] < 1e-12 * S[0]
    assert np.min(-np.diff(S[:k])) > 1e-2 * S[0]
    return D, rows, cols


def _topk(D, k):
    U, S, Vt = np.linalg.svd(D, full_matrices=False)
    return U[:, :k], S[:k], Vt[:k].T


def _loss_terms(k, m, n, seed):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((m, k))
    Dd = rng.standard_normal((n, k))
    w = rng.random(k) + 0.5
    w2 = rng.random(k) + 0.5
    W = rng.standard_normal((k, 3))

    def loss(U, S, V):
        return (S.sum() + (w * ((C * U).sum(0)) ** 2).sum()
                + (w2 * ((Dd * V).sum(0)) ** 2).sum() + np.sum((U @ W) ** 2))

    def grads(U, S, V):
        dU = 2 * C * (w * (C * U).sum(0))[None, :] + 2 * U @ W @ W.T
        dV = 2 * Dd * (w2 * (Dd * V).sum(0))[None, :]
        return dU, np.ones(k), dV

    return loss, grads


def _fd(D, rows, cols, k, lossfn, idx, rel_h=1e-6):
    out = np.empty(len(idx))
    for t, e in enumerate(idx):
        r, c = rows[e], cols[e]
        h = rel_h * max(abs(D[r, c]), 0.05)
        Dp = D.copy()
        Dp[r, c] += h
        Dm = D.copy()
        Dm[r, c] -= h
        out[t] = (lossfn(*_topk(Dp, k)) - lossfn(*_topk(Dm, k))) / (2 * h)
    return out


def test_adjoint_matches_fd_on_exact_rank_input():
    m, n, k = 30, 20, 4
    D, rows, cols = _exact_rank_pattern(m, n, k, seed=3)
    loss, grads = _loss_terms(k, m, n, seed=4)
    U, S, V = _topk(D, k)
    dU, dS, dV = grads(U, S, V)
    g = oracle.svd_adjoint_values(U, S, V, dU, dS, dV, rows, cols)
    fd = _fd(D, rows, cols, k, loss, range(rows.size))
    assert np.abs(g - fd).max() < 1e-5 * np.abs(fd).max()


def test_adjoint_sigma_sum_closed_form_and_fd():
    # d(sum sigma_i)/dA = U_k V_k^T, exact for any k with sigma_k > sigma_{k+1}
    D = np.random.default_rng(5).standard_normal((25, 18)) * (np.random.default_rng(6).random((25, 18)) < 0.4)
    rows, cols = np.nonzero(D)
    k = 6
    U, S, V = _topk(D, k)
    g = oracle.svd_adjoint_values(U, S, V, None, np.ones(k), None, rows, cols)
    closed = (U[rows] * V[cols]).sum(1)
    np.testing.assert_allclose(g, closed, atol=1e-13)
    fd = _fd(D, rows, cols, k, lambda U, S, V: S.sum(), range(0, rows.size, 7))
    np.testing.assert_allclose(g[::7], fd, atol=1e-6)


def test_adjoint_invariant_term_is_zero():
    D = np.random.default_rng(7).standard_normal((20, 15))
    rows, cols = np.nonzero(D)
    k = 5
    U, S, V = _topk(D, k)
    W = np.random.default_rng(8).standard_normal((k, 8))
    dU = 2 * U @ W @ W.T
    g = oracle.svd_adjoint_values(U, S, V, dU, None, None, rows, cols)
    assert np.abs(g).max() < 1e-12
    fd = _fd(D, rows, cols, k, lambda U, S, V: np.sum((U @ W) ** 2), range(0, rows.size, 11))
    assert np.abs(fd).max() < 1e-6


def test_adjoint_slice_of_differentiated_workload():
    # the 300 x 200 corner of the 500K x 100K Zipf workload as its own input, k = 50, with
    # the loss sum(sigma) + ||U_k W||^2 (W 50 x 8): the second term is invariant, so the
    # adjoint is exact and finite differences of the exact-SVD loss must match it
    A = zipf_normal(m=2000, n=100_000)
    D = A.toarray()[:300, :200]
    rows, cols = np.nonzero(D)
    assert 2000 < rows.size < 8000
    k = 50
    W = np.random.default_rng(7).standard_normal((k, 8))
    U, S, V = _topk(D, k)
    g = oracle.svd_adjoint_values(U, S, V, 2 * U @ W @ W.T, np.ones(k), None, rows, cols)
    idx = np.random.default_rng(9).choice(rows.size, 60, replace=False)
    fd = _fd(D, rows, cols, k, lambda U, S, V: S.sum() + np.sum((U @ W) ** 2), idx)
    np.testing.assert_allclose(g[idx], fd, atol=2e-5)


@pytest.mark.parametrize("flip", ["J", "K", "F"])
def test_planted_mistakes_are_caught(flip):
    # A mistake planted in a copy of the formula must fail the finite-difference check.
    m, n, k = 30, 20, 4
    D, rows, cols = _exact_rank_pattern(m, n, k, seed=3)
    loss, grads = _loss_terms(k, m, n, seed=4)
    U, S, V = _topk(D, k)
    dU, dS, dV = grads(U, S, V)
    J = U.T @ dU
    K = V.T @ dV
    s2 = S ** 2
    Dm = s2[None, :] - s2[:, None]
    F = np.zeros((k, k))
    off = ~np.eye(k, dtype=bool)
    F[off] = 1.0 / Dm[off]
    if flip == "F":
        F = -F
    Jt = J.T if flip != "J" else -J.T
    Kt = K.T if flip != "K" else -K.T
    M = (F * (J - Jt)) * S[None, :] + np.diag(dS) + S[:, None] * (F * (K - Kt))
    Ab = U @ M @ V.T + (dU - U @ J) / S @ V.T + (U / S) @ (dV - V @ K).T
    bad = Ab[rows, cols]
    fd = _fd(D, rows, cols, k, loss, range(rows.size))
    assert np.abs(bad - fd).max() > 1e-3 * np.abs(fd).max()
