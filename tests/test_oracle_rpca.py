"""Pins of the FP64 basic randomized PCA (Alg. 1 and Alg. 4) against the paper's theorems and
against references that share none of its code.

* Theorem 1 (Alg. 5 with even q equals Alg. 1 with p = (q - 2) / 2) and Theorem 2 (Alg. 6
  with even q equals Alg. 4) on the same Gaussian draws: the fast oracle builds its bases by
  LU and eigSVD, the basic one by Householder QR, so a mistake in either breaks the equality.
* A full subspace (l = min(m, n)) makes both algorithms exact for any p: compared with the
  from-scratch one-sided Jacobi SVD.
* rank(A) <= k: exact recovery of the nonzero triplets, the rest reported as zero.
* Power steps converge: on a planted spectrum the error of sigma_k shrinks with p.
* Planted mistakes (a dropped power step, the other sketch side, U and V exchanged) each
  fail one of these checks.
"""
import numpy as np
import pytest

import oracle
from oracle.rpca import rpca
from refs import jacobi_svd, sigma_rel_err, sin_theta
from synth import planted_blocks, random_sparse


def _tall():
    return random_sparse(80, 45, 0.3, seed=21)


def _wide():
    return random_sparse(45, 80, 0.3, seed=22)


@pytest.mark.parametrize("q", [2, 4, 6, 8])
def test_theorem1_alg5_equals_alg1(q):
    A = _wide()
    k, s, seed = 8, 4, 98
    U, S, V, info = oracle.frpca(A, k, q, s, seed)
    assert info["orientation"] == "alg5"
    Ur, Sr, Vr = rpca(A, k, (q - 2) // 2, s, seed, alg=1)
    assert sigma_rel_err(Sr, S) < 1e-10
    assert sin_theta(Ur, U) < 1e-8 and sin_theta(Vr, V) < 1e-8
    # the sign convention makes the factors equal, not only their ranges
    assert np.abs(Ur - U).max() < 1e-8 and np.abs(Vr - V).max() < 1e-8


@pytest.mark.parametrize("q", [2, 4, 6, 8])
def test_theorem2_alg6_equals_alg4(q):
    A = _tall()
    k, s, seed = 8, 4, 99
    U, S, V, info = oracle.frpca(A, k, q, s, seed)
    assert info["orientation"] == "alg6"
    Ur, Sr, Vr = rpca(A, k, (q - 2) // 2, s, seed, alg=4)
    assert sigma_rel_err(Sr, S) < 1e-10
    assert np.abs(Ur - U).max() < 1e-8 and np.abs(Vr - V).max() < 1e-8


@pytest.mark.parametrize("alg", [1, 4])
@pytest.mark.parametrize("p", [0, 1, 3])
@pytest.mark.parametrize("shape", [(14, 9), (9, 14)])
def test_full_subspace_is_exact_svd(alg, p, shape):
    A = random_sparse(*shape, 0.6, seed=31)
    l = min(shape)
    k, s = l - 3, 3
    U, S, V = rpca(A, k, p, s, seed=3, alg=alg)
    Uj, Sj, Vj = jacobi_svd(A.toarray())
    np.testing.assert_allclose(S, Sj[:k], rtol=1e-10)
    for i in range(k):
        assert abs(abs(U[:, i] @ Uj[:, i]) - 1) < 1e-9
        assert abs(abs(V[:, i] @ Vj[:, i]) - 1) < 1e-9


@pytest.mark.parametrize("alg", [1, 4])
@pytest.mark.parametrize("tall", [True, False])
def test_exact_recovery_rank_le_k(alg, tall):
    P = planted_blocks(m=60, n=40, blocks=4, seed=41, decades=1.0)
    A = P if tall else oracle.transpose(P)
    k, s = 6, 3
    U, S, V = rpca(A, k, 1, s, seed=8, alg=alg)
    Dn = P.toarray() if tall else P.toarray().T
    sig_true = np.linalg.svd(Dn, compute_uv=False)
    np.testing.assert_allclose(S[:4], sig_true[:4], rtol=1e-10)
    assert np.all(S[4:] == 0) and np.all(U[:, 4:] == 0) and np.all(V[:, 4:] == 0)
    np.testing.assert_allclose((U[:, :4] * S[:4]) @ V[:, :4].T, Dn, atol=10 * sig_true[4] + 1e-14)


@pytest.mark.parametrize("alg", [1, 4])
def test_power_steps_converge_on_planted_spectrum(alg):
    P = planted_blocks(m=3000, n=1200, blocks=60, seed=42)
    sig = np.linalg.svd(P.toarray(), compute_uv=False)
    k, s = 20, 5
    errs = []
    for p in (0, 1, 2):
        U, S, V = rpca(P, k, p, s, seed=5, alg=alg)
        assert np.all(S <= sig[:k] * (1 + 1e-12))           # Rayleigh-Ritz values interlace
        errs.append(float(np.max((sig[:k] - S) / sig[:k])))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.1 * errs[0]


def test_planted_mistakes_are_caught():
    A = _tall()
    k, s, seed, q = 8, 4, 99, 6
    U, S, V, _ = oracle.frpca(A, k, q, s, seed)
    # one power step too few: no longer Theorem 2's partner
    Ur, Sr, Vr = rpca(A, k, (q - 2) // 2 - 1, s, seed, alg=4)
    assert sigma_rel_err(Sr, S) > 1e-6
    # Alg. 1 on a tall matrix is a different sketch (same p), not Alg. 6's partner
    Ur, Sr, Vr = rpca(A, k, (q - 2) // 2, s, seed, alg=1)
    assert sigma_rel_err(Sr, S) > 1e-6
    # U and V exchanged: shapes differ, so compare ranges on the square case
    B = random_sparse(30, 30, 0.4, seed=5)
    U1, S1, V1 = rpca(B, 6, 1, 3, seed=2, alg=4)
    U0, S0, V0, _ = oracle.frpca(B, 6, 4, 3, seed=2)
    assert sin_theta(U0, U1) < 1e-8
    assert sin_theta(U0, V1) > 1e-3


def test_argument_rules():
    A = _tall()
    for kw in ({"k": 0, "p": 1, "s": 2}, {"k": 40, "p": 1, "s": 10}, {"k": 4, "p": -1, "s": 2}):
        with pytest.raises(ValueError):
            rpca(A, kw["k"], kw["p"], kw["s"], seed=1, alg=1)
    with pytest.raises(ValueError):
        rpca(A, 4, 1, 2, seed=1, alg=2)
