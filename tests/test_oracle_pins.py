"""Pins of the FP64 oracle against the paper's lemmas/theorems and independent references.

Every check compares the oracle with something other than itself: published known-answer
vectors, a dense BLAS/LAPACK computation of a different routine, a from-scratch Jacobi SVD,
the textbook randomized SVD of Alg. 1 / Alg. 4 (Theorems 1 and 2), closed-form planted
spectra, or invariants (Rayleigh-Ritz interlacing, Lemma 3's range equality).
"""
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

import oracle
from refs import (jacobi_svd, orth_err, rpca_basic, rpcat_basic, sigma_rel_err, sin_theta,
                  subspace_iteration)
from synth import from_dense, planted_blocks, random_sparse, small_decay


# ---------------------------------------------------------------- Philox / Gaussian draws
def _kat_rows(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_known_answers(golden_dir):
    rows = _kat_rows(golden_dir)
    assert len(rows) == 3
    for r in rows:
        out = oracle.philox4x32_10(*r[:6])
        assert [int(x) for x in out] == r[6:]


def test_philox_stream_layout():
    # block b uses counter (b mod 2^32, b div 2^32, 0, 0) and key (seed lo, seed hi)
    seed = 0x0123456789ABCDEF
    w = oracle.uint32_stream(seed, 3, first_block=(1 << 32) - 1)
    for i, b in enumerate(range((1 << 32) - 1, (1 << 32) + 2)):
        ref = oracle.philox4x32_10(b & 0xFFFFFFFF, b >> 32, 0, 0, seed & 0xFFFFFFFF, seed >> 32)
        assert [int(x) for x in ref] == [int(x) for x in w[i]]


def test_gaussian_distribution():
    z = oracle.gaussian(20181015, 500, 400).ravel()
    assert abs(z.mean()) < 5e-3
    assert abs(z.var() - 1) < 1e-2
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # uniform words pass a chi-square test on 256 bins of the top byte
    w = oracle.uint32_stream(7, 100_000).ravel() >> 24
    counts = np.bincount(w.astype(np.int64), minlength=256)
    assert scipy.stats.chisquare(counts).pvalue > 1e-3


def test_gaussian_element_indexing():
    # element [r, j] of a rows x cols draw is normal number r*cols + j of the stream
    g = oracle.gaussian(11, 7, 5)
    flat = oracle.gaussian(11, 1, 35).ravel()
    assert np.array_equal(g.ravel(), flat)
    assert np.array_equal(oracle.gaussian(11, 3, 5), g[:3])


# ---------------------------------------------------------------- sparse products / mirror
def test_spmm_matches_dense():
    A = random_sparse(70, 45, 0.1, seed=3, empty_rows=(0, 13), empty_cols=(5,))
    D = A.toarray()
    X = np.random.default_rng(0).standard_normal((45, 9))
    Y = np.random.default_rng(1).standard_normal((70, 9))
    np.testing.assert_allclose(oracle.csr_matmul(A, X), D @ X, rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.csr_tmatmul(A, Y), D.T @ Y, rtol=0, atol=1e-12)


def test_csc_mirror_matches_scipy():
    A = random_sparse(90, 60, 0.08, seed=4, empty_rows=(2,), empty_cols=(0, 59))
    col_ptr, row, perm = oracle.csc_mirror(A)
    C = A.to_scipy().tocsc()
    C.sort_indices()
    assert np.array_equal(col_ptr, C.indptr)
    assert np.array_equal(row, C.indices)
    np.testing.assert_array_equal(A.val[perm].astype(np.float64), C.data)
    assert np.array_equal(np.sort(perm), np.arange(A.nnz))


# ---------------------------------------------------------------- LU basis (Lemma 3)
def test_lu_matches_lapack_partial_pivoting():
    X = np.random.default_rng(5).standard_normal((200, 12))
    L, piv, dropped = oracle.lu_pl(X)
    P, Ls, Us = scipy.linalg.lu(X)        # X = P Ls Us, so P^T L of the paper is P @ Ls
    assert dropped == []
    np.testing.assert_allclose(L, P @ Ls, rtol=0, atol=1e-12)
    # pivot rows in pivot order form a unit lower-triangular block, and |L| <= 1
    np.testing.assert_allclose(L[piv], np.tril(L[piv]), atol=0)
    np.testing.assert_allclose(np.diag(L[piv]), 1.0, atol=0)
    assert np.abs(L).max() <= 1.0 + 1e-15
    # P^T L spans range(X) (Lemma 3)
    Qx = np.linalg.qr(X)[0]
    Ql = np.linalg.qr(L)[0]
    assert sin_theta(Qx, Ql) < 1e-12
    # and X = P^T L U with U from the pivot rows
    U = np.linalg.solve(L[piv], X[piv])
    np.testing.assert_allclose(L @ U, X, atol=1e-12)


def test_lu_rank_guard():
    rng = np.random.default_rng(6)
    X = rng.standard_normal((150, 4)) @ rng.standard_normal((4, 9))   # rank 4 of 9
    L, piv, dropped = oracle.lu_pl(X)
    assert len(dropped) == 5 and len(piv) == 4
    assert np.all(L[:, dropped] == 0)
    Qx = np.linalg.svd(X, full_matrices=False)[0][:, :4]
    kept = [j for j in range(9) if j not in dropped]
    assert sin_theta(Qx, np.linalg.qr(L[:, kept])[0]) < 1e-10
    assert sin_theta(np.linalg.qr(L[:, kept])[0], Qx) < 1e-10


def test_lu_tie_goes_to_lowest_row():
    X = np.array([[1.0, 2.0], [-3.0, 1.0], [3.0, 5.0], [0.5, 0.0]])
    L, piv, _ = oracle.lu_pl(X)
    assert piv[0] == 1


# ---------------------------------------------------------------- eigSVD (Alg. 2, Lemma 1)
def test_eig_ascending_residual():
    B = np.random.default_rng(7).standard_normal((30, 30))
    B = B @ B.T
    d, V = oracle.eig_asc(B)
    assert np.all(np.diff(d) >= 0)
    assert np.abs(B @ V - V * d).max() < 1e-12 * np.abs(d).max()
    assert orth_err(V) < 1e-13


def test_eigsvd_is_economic_svd_lemma1():
    X = np.random.default_rng(8).standard_normal((300, 14)) @ np.diag(np.linspace(1, 6, 14))
    U, S, V, nd = oracle.eigsvd(X)
    assert nd == 0 and np.all(np.diff(S) > 0)          # ascending
    Ur, Sr, Vrt = np.linalg.svd(X, full_matrices=False)
    np.testing.assert_allclose(S[::-1], Sr, rtol=1e-12)
    for j in range(14):  # columns agree up to a common sign
        sgn = np.sign(V[:, ::-1][:, j] @ Vrt[j])
        np.testing.assert_allclose(U[:, ::-1][:, j] * sgn, Ur[:, j], atol=1e-10)
    np.testing.assert_allclose((U * S) @ V.T, X, atol=1e-11)


def test_eigsvd_against_jacobi_svd():
    X = np.random.default_rng(9).standard_normal((25, 8))
    U, S, V, _ = oracle.eigsvd(X)
    Uj, Sj, Vj = jacobi_svd(X)
    np.testing.assert_allclose(S[::-1], Sj, rtol=1e-12)
    assert sin_theta(Uj[:, :3], U[:, ::-1][:, :3]) < 1e-10


def test_eigsvd_rank_guard():
    rng = np.random.default_rng(10)
    X = rng.standard_normal((80, 3)) @ rng.standard_normal((3, 7))
    # eigSVD's noise floor is ~sqrt(eps) * sigma_max, so the guard must sit above it
    U, S, V, nd = oracle.eigsvd(X, tol=1e-6)
    assert nd == 4 and np.all(S[:4] == 0) and np.all(U[:, :4] == 0)
    Sr = np.linalg.svd(X, compute_uv=False)
    np.testing.assert_allclose(S[4:][::-1], Sr[:3], rtol=1e-12)


def test_jacobi_reference_itself_against_lapack():
    A = np.random.default_rng(11).standard_normal((9, 13))
    U, s, V = jacobi_svd(A)
    np.testing.assert_allclose(s, np.linalg.svd(A, compute_uv=False), rtol=1e-13)
    np.testing.assert_allclose((U * s) @ V.T, A, atol=1e-13)


# ---------------------------------------------------------------- frPCA (Alg. 5 / Alg. 6)
def _tall():
    return random_sparse(90, 50, 0.3, seed=21)


def _wide():
    return random_sparse(45, 80, 0.3, seed=22)


@pytest.mark.parametrize("q", [2, 4, 6])
def test_theorem2_alg6_equals_basic_rpcat(q):
    A = _tall()
    k, s, seed = 8, 4, 99
    U, S, V, info = oracle.frpca(A, k, q, s, seed, sign_fix=False)
    assert info["orientation"] == "alg6"
    omega_lm = oracle.gaussian(seed, A.m, k + s).T      # randn(k+s, m)
    Ur, Sr, Vr = rpcat_basic(A.toarray(), k, (q - 2) // 2, omega_lm)
    assert sigma_rel_err(Sr, S) < 1e-10
    assert sin_theta(Ur, U) < 1e-8 and sin_theta(Vr, V) < 1e-8


@pytest.mark.parametrize("q", [2, 4, 6])
def test_theorem1_alg5_equals_basic_rpca(q):
    A = _wide()
    k, s, seed = 8, 4, 98
    U, S, V, info = oracle.frpca(A, k, q, s, seed, sign_fix=False)
    assert info["orientation"] == "alg5"
    omega = oracle.gaussian(seed, A.n, k + s)             # randn(n, k+s)
    Ur, Sr, Vr = rpca_basic(A.toarray(), k, (q - 2) // 2, omega)
    assert sigma_rel_err(Sr, S) < 1e-10
    assert sin_theta(Ur, U) < 1e-8 and sin_theta(Vr, V) < 1e-8


@pytest.mark.parametrize("q", [3, 5, 7])
def test_odd_passes_equal_subspace_iteration(q):
    for A, right in ((_tall(), True), (_wide(), False)):
        k, s, seed = 7, 5, 97
        U, S, V, _ = oracle.frpca(A, k, q, s, seed, sign_fix=False)
        rows = A.n if right else A.m
        omega = oracle.gaussian(seed, rows, k + s)
        Ur, Sr, Vr = subspace_iteration(A.toarray(), k, (q - 1) // 2, omega, right=right)
        assert sigma_rel_err(Sr, S) < 1e-10
        assert sin_theta(Ur, U) < 1e-8 and sin_theta(Vr, V) < 1e-8


@pytest.mark.parametrize("q", [2, 3, 4, 5, 6, 7, 8])
def test_pass_schedule_spends_exactly_q_passes(q):
    """q is the number of passes over A (Section 3.3): counting the products the routine
    makes gives q; LU bases come before the one eigSVD basis, and an even q starts with a
    product of the long-side Gaussian matrix."""
    D = np.random.default_rng(q).standard_normal((40, 25))
    calls = []

    def fwd(X):
        calls.append("fwd")
        return D @ X

    def back(Y):
        calls.append("back")
        return D.T @ Y

    oracle.randomized_svd(fwd, back, 40, 25, 4, q, 3, seed=1)
    assert len(calls) == q
    assert calls[0] == ("back" if q % 2 == 0 else "fwd")
    assert calls[-1] == "fwd"
    start, bases = oracle.pass_schedule(q)
    assert start == ("sketch" if q % 2 == 0 else "gaussian")
    assert bases.count("eig") == 1 and bases[-1] == "eig"
    assert len(bases) == (q - 1) // 2 + (q % 2 == 0)


@pytest.mark.parametrize("q", [2, 3, 5])
@pytest.mark.parametrize("shape", [(14, 9), (9, 14)])
def test_full_subspace_is_exact_svd(q, shape):
    A = random_sparse(*shape, 0.6, seed=31)
    l = min(shape)
    k, s = l - 3, 3
    U, S, V, _ = oracle.frpca(A, k, q, s, seed=3)
    Uj, Sj, Vj = jacobi_svd(A.toarray())
    np.testing.assert_allclose(S, Sj[:k], rtol=1e-10)
    for i in range(k):
        assert abs(abs(U[:, i] @ Uj[:, i]) - 1) < 1e-9
        assert abs(abs(V[:, i] @ Vj[:, i]) - 1) < 1e-9


@pytest.mark.parametrize("q", [2, 3, 4, 7])
@pytest.mark.parametrize("tall", [True, False])
def test_exact_recovery_rank_le_k(q, tall):
    P = planted_blocks(m=60, n=40, blocks=4, seed=41, decades=1.0)
    A = P if tall else oracle.transpose(P)
    k, s = 6, 3
    U, S, V, info = oracle.frpca(A, k, q, s, seed=8)
    sig = P.meta["sigma"]
    Dn = A.toarray() if tall else P.toarray().T
    sig_true = np.linalg.svd(Dn, compute_uv=False)
    np.testing.assert_allclose(S[:4], sig_true[:4], rtol=1e-10)
    np.testing.assert_allclose(S[:4], sig, rtol=1e-6)   # float32-rounded values
    assert np.all(S[4:] == 0) and info["rank_dropped"] == 2
    assert np.all(U[:, 4:] == 0) and np.all(V[:, 4:] == 0)
    # the float32 rounding of the planted values leaves sigma_5.. ~ 3e-9 in A itself
    tail = sig_true[4]
    np.testing.assert_allclose((U[:, :4] * S[:4]) @ V[:, :4].T, Dn, atol=10 * tail + 1e-14)


def test_planted_spectrum_interlacing_and_convergence():
    P = planted_blocks(m=3000, n=1200, blocks=60, seed=42)
    sig = np.linalg.svd(P.toarray(), compute_uv=False)
    np.testing.assert_allclose(sig[:60], P.meta["sigma"], rtol=1e-6)
    k, s = 10, 5
    errs = []
    for q in (2, 3, 5, 9):
        U, S, V, _ = oracle.frpca(P, k, q, s, seed=1)
        assert np.all(S <= sig[:k] * (1 + 1e-12))   # Rayleigh-Ritz values never exceed sigma_i
        assert orth_err(U) < 1e-12 and orth_err(V) < 1e-12
        errs.append(sigma_rel_err(sig[:k], S))
    # more passes converge further (sigma_10/sigma_16 = 0.5 here, so q = 9 reaches ~1e-4)
    assert all(b < a for a, b in zip(errs, errs[1:])) and errs[-1] < 1e-3


def test_small_decay_workload_accuracy_and_identities():
    A = small_decay()
    U, S, V, info = oracle.frpca(A, 10, 3, 5, seed=20181015)
    D = A.toarray()
    sig = np.linalg.svd(D, compute_uv=False)
    assert info["orientation"] == "alg6"
    assert np.all(S <= sig[:10] * (1 + 1e-12))
    # three passes: the leading values are close, the tail of the k is still converging
    assert sigma_rel_err(sig[:5], S[:5]) < 0.02 and sigma_rel_err(sig[:10], S) < 0.2
    # the Gram-based eigSVD basis loses orthogonality like u * cond(X)^2
    assert orth_err(U) < 1e-10 and orth_err(V) < 1e-10
    np.testing.assert_allclose(D @ V, U * S, atol=1e-12)   # U = A V S^-1 by construction
    U11, S11, V11, _ = oracle.frpca(A, 10, 11, 5, seed=20181015)
    # eleven passes: the leading values are converged to rounding, the 10th to ~2e-5
    assert sigma_rel_err(sig[:10], S11) < 1e-4 and sigma_rel_err(sig[:4], S11[:4]) < 1e-12


def test_sign_convention():
    A = _tall()
    U, S, V, _ = oracle.frpca(A, 5, 4, 3, seed=2)
    for i in range(5):
        j = np.argmax(np.abs(V[:, i]))
        assert V[j, i] > 0


def test_argument_rules():
    A = _tall()
    with pytest.raises(ValueError):
        oracle.frpca(A, 5, 1, 3, seed=1)      # q = 1 is rejected (Alg. 5/6 need q >= 2)
    with pytest.raises(ValueError):
        oracle.frpca(A, 45, 3, 6, seed=1)     # k + s > min(m, n)
    with pytest.raises(ValueError):
        oracle.frpca(A, 0, 3, 6, seed=1)


def test_dense_input_roundtrip():
    D = np.zeros((5, 4))
    D[0, 1] = 2.0
    D[3, 0] = -1.0
    A = from_dense(D)
    U, S, V, info = oracle.frpca(A, 2, 2, 1, seed=0)
    np.testing.assert_allclose(S, [2.0, 1.0], rtol=1e-12)
