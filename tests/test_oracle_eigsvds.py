"""Pins of the FP64 eigSVDs (Alg. 3) against routines that share none of its code.

* It is the truncated SVD: compared with LAPACK's SVD of the dense matrix (a different
  routine than the symmetric eigensolver it calls), for tall and wide inputs.
* Tiny matrices: compared with the from-scratch one-sided Jacobi SVD.
* Planted block spectrum: the closed-form singular values; rank below k gives zeros.
* Planted mistakes (eigenvalues in ascending order, U without the 1/S scaling, the larger
  Gram matrix's orientation swapped) each fail one of these checks.
"""
import numpy as np
import pytest

import oracle
from oracle.eigsvds import eigsvds
from refs import jacobi_svd, sin_theta
from synth import planted_blocks, random_sparse


@pytest.mark.parametrize("shape", [(400, 60), (60, 400), (300, 300)])
def test_equals_truncated_svd(shape):
    A = random_sparse(*shape, 0.08, seed=sum(shape))
    k = 12
    U, S, V = eigsvds(A, k)
    Ud, Sd, Vdt = np.linalg.svd(A.toarray(), full_matrices=False)
    np.testing.assert_allclose(S, Sd[:k], rtol=1e-10)
    for i in range(k):
        gap = min(abs(Sd[i] - Sd[i + 1]), abs(Sd[i] - Sd[i - 1]) if i else np.inf) / Sd[0]
        if gap > 1e-3:
            assert abs(abs(U[:, i] @ Ud[:, i]) - 1) < 1e-8
            assert abs(abs(V[:, i] @ Vdt[i]) - 1) < 1e-8
    # A V = U diag(S) and orthonormal factors
    assert np.abs(A.toarray() @ V - U * S).max() < 1e-10 * S[0]
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-10 and np.abs(V.T @ V - np.eye(k)).max() < 1e-12


@pytest.mark.parametrize("shape", [(30, 20), (20, 30)])
def test_against_jacobi_svd(shape):
    A = random_sparse(*shape, 0.5, seed=3)
    k = 8
    U, S, V = eigsvds(A, k)
    Uj, Sj, Vj = jacobi_svd(A.toarray())
    np.testing.assert_allclose(S, Sj[:k], rtol=1e-11)
    assert sin_theta(Uj[:, :k], U) < 1e-8 and sin_theta(Vj[:, :k], V) < 1e-8


def test_planted_closed_form_and_rank():
    P = planted_blocks(m=3000, n=800, blocks=40, seed=9)
    U, S, V = eigsvds(P, 30)
    np.testing.assert_allclose(S, P.meta["sigma"][:30], rtol=1e-6)   # float32-rounded values
    Q = planted_blocks(m=300, n=120, blocks=6, seed=10, decades=1.0)
    U, S, V = eigsvds(Q, 9)
    assert np.all(S[6:] == 0) and np.all(U[:, 6:] == 0) and np.all(V[:, 6:] == 0)
    np.testing.assert_allclose(S[:6], Q.meta["sigma"], rtol=1e-6)
    # sign convention
    piv = np.argmax(np.abs(V[:, :6]), axis=0)
    assert np.all(V[piv, np.arange(6)] > 0)


def test_planted_mistakes_are_caught():
    A = random_sparse(200, 50, 0.1, seed=4)
    k = 6
    sp = A.to_scipy()
    d, W = np.linalg.eigh((sp.T @ sp).toarray())
    Sd = np.linalg.svd(A.toarray(), compute_uv=False)[:k]
    # the k smallest eigenvalues instead of the largest
    assert np.max(np.abs(np.sqrt(np.maximum(d[:k][::-1], 0)) - Sd) / Sd) > 0.1
    # U = A V without 1/S is not orthonormal
    V = W[:, ::-1][:, :k]
    Ubad = sp @ V
    assert np.abs(Ubad.T @ Ubad - np.eye(k)).max() > 1e-3
    # the oracle itself passes the same checks
    U, S, V2 = eigsvds(A, k)
    assert np.abs(U.T @ U - np.eye(k)).max() < 1e-10
    np.testing.assert_allclose(S, Sd, rtol=1e-10)


def test_argument_rules():
    A = random_sparse(40, 20, 0.3, seed=1)
    for k in (0, 21):
        with pytest.raises(ValueError):
            eigsvds(A, k)
