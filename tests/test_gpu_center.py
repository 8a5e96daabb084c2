"""Centred mode on the GPU (opts.center: principal components of A - 1 mu^T, mu = column
means of A, never formed) against the FP64 oracle's centred mode on the same Gaussian draws.

Tolerances as for the uncentred path: relative singular-value error <= 1e-4 and largest
principal angle <= 1e-3 rad on the separable leading block; the backward against the oracle's
centred adjoint evaluated at the GPU's own factors.
"""
import numpy as np
import pytest

import oracle
from gpu_util import compare_triplets, np64, say
from synth import random_sparse, small_decay, zipf_lognormal, zipf_normal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1810_06825_amd import FrPCA  # noqa: E402

DEV = "cuda:0"


def _check(A, k, q, s, seed, **kw):
    say("centred frpca", A.m, A.n, A.nnz, f"k={k} q={q} s={s}", kw)
    mat = FrPCA.from_csr(A, device=DEV, center=True, **kw)
    U, S, V = mat.run(k, q, s, seed)
    torch.cuda.synchronize()
    Ug, Sg, Vg = np64(U), np64(S), np64(V)
    Uo, So, Vo, _ = oracle.frpca(A, k, q, s, seed, center=True)
    S_ritz = oracle.frpca(A, k + 1, q, s - 1, seed, center=True)[1]
    r = compare_triplets(Uo, So, Vo, Ug, Sg, Vg, S_ritz)
    say("  ->", {kk: (round(v, 8) if isinstance(v, float) else v) for kk, v in r.items()})
    return r, mat, (U, S, V)


@pytest.mark.parametrize("q", [3, 4, 5])
def test_centred_tall(q):
    A = zipf_lognormal(m=30_011, n=4_003, t=40)
    r, mat, (U, S, V) = _check(A, 20, q, 10, 500 + q)
    assert r["ok"], r
    # component scores have zero column means; the centred spectrum differs from A's
    Ug = np64(U)
    assert np.abs(Ug.sum(axis=0)).max() < 1e-4 * np.sqrt(A.m)
    U0, S0, V0 = FrPCA.from_csr(A, device=DEV).run(20, q, 10, 500 + q)
    assert abs(float(S0[0]) - float(S[0])) > 1e-3 * float(S0[0])
    mat.close()


@pytest.mark.parametrize("q", [2, 3, 5])
def test_centred_wide_alg5(q):
    A = zipf_normal(m=3_001, n=20_011, t=30)
    r, mat, _ = _check(A, 16, q, 8, 700 + q)
    assert r["ok"], r
    mat.close()


def test_centred_small_decay_and_set_values():
    A = small_decay()
    r, mat, _ = _check(A, 10, 3, 5, 20181015)
    assert r["ok"] and r["prefix"] >= 8
    # new values: the column means follow (against a fresh handle and the oracle)
    rng = np.random.default_rng(5)
    v2 = (A.val * (1.0 + 0.5 * rng.random(A.nnz))).astype(np.float32)
    mat.set_values(torch.from_numpy(v2).to(DEV))
    U1, S1, V1 = mat.run(10, 3, 5, 20181015)
    A2 = type(A)(A.m, A.n, A.row_ptr, A.col, v2, dict(A.meta))
    U2, S2, V2 = FrPCA.from_csr(A2, device=DEV, center=True).run(10, 3, 5, 20181015)
    assert torch.equal(S1, S2) and torch.equal(U1, U2) and torch.equal(V1, V2)
    So = oracle.frpca(A2, 10, 3, 5, 20181015, center=True)[1]
    assert np.max(np.abs(np64(S1) - So) / So) < 1e-4
    mat.close()


@pytest.mark.parametrize("k", [12, 13])
def test_centred_backward_matches_fp64_formula(k):
    # k = 12 runs the paired SDDMM, k = 13 the two-column form
    A = random_sparse(4_000, 900, 0.02, seed=77)
    mat = FrPCA.from_csr(A, device=DEV, center=True)
    U, S, V = mat.run(k, 4, 8, 31)
    rng = np.random.default_rng(3)
    dU = torch.from_numpy(rng.standard_normal((A.m, k)).astype(np.float32)).to(DEV)
    dV = torch.from_numpy(rng.standard_normal((A.n, k)).astype(np.float32)).to(DEV)
    dS = torch.ones(k, device=DEV)
    say("centred backward", A.m, A.n, A.nnz, k)
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    # without dV the sampled product has one term (its own kernel variant)
    g1 = np64(mat.backward(dU, dS, None))
    ref1 = oracle.svd_adjoint_values(np64(U), np64(S), np64(V), np64(dU), np64(dS), None, rows, A.col,
                                     center=True)
    err1 = np.abs(g1 - ref1).max() / np.abs(ref1).max()
    say("  rel err without dV", err1)
    assert err1 < 1e-4
    g = np64(mat.backward(dU, dS, dV))
    assert np.abs(np64(mat.adjoint(U, S, V, dU, dS, dV)) - g).max() <= 1e-6 * np.abs(g).max()
    ref = oracle.svd_adjoint_values(np64(U), np64(S), np64(V), np64(dU), np64(dS), np64(dV), rows, A.col,
                                    center=True)
    err = np.abs(g - ref).max() / np.abs(ref).max()
    say("  rel err", err)
    assert err < 1e-4
    # the uncentred adjoint is far from what the GPU returns (the centring term is resolved)
    ref0 = oracle.svd_adjoint_values(np64(U), np64(S), np64(V), np64(dU), np64(dS), np64(dV), rows, A.col)
    assert np.abs(ref0 - ref).max() / np.abs(ref).max() > max(1e-4, 100 * err)
    mat.close()


def test_centred_bf16_panels():
    A = zipf_lognormal(m=30_011, n=4_003, t=40)
    mat = FrPCA.from_csr(A, device=DEV, center=True, panel_bf16=True)
    U, S, V = mat.run(20, 5, 10, 11)
    So = oracle.frpca(A, 20, 5, 10, 11, center=True)[1]
    err = float(np.max(np.abs(np64(S) - So) / So))
    say("centred bf16 sigma err", err)
    assert err < 2e-3
    mat.close()
