"""eigSVDs (Alg. 3) on the GPU against the FP64 oracle (dense B = A^T A and LAPACK's
eigensolver), through the C-ABI: tall and wide inputs, a planted spectrum against its closed
form, repeatability, the iteration limit and argument errors.
"""
import numpy as np
import pytest

import oracle
from gpu_util import ANG_TOL, SIG_TOL, compare_triplets, np64, say
from synth import aminer_tfidf, planted_blocks, zipf_lognormal, zipf_normal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1810_06825_amd import FrPCA, FrpcaError, binding  # noqa: E402

DEV = "cuda:0"


def _check(A, k, s, seed=11):
    say("eigsvds", A.meta.get("workload", "matrix"), A.m, A.n, A.nnz, f"k={k} s={s}")
    mat = FrPCA.from_csr(A, device=DEV)
    U, S, V, it = mat.eigsvds(k, s, seed)
    U2, S2, V2, it2 = mat.eigsvds(k, s, seed)
    assert torch.equal(U, U2) and torch.equal(S, S2) and torch.equal(V, V2) and it == it2
    mat.close()
    Ug, Sg, Vg = np64(U), np64(S), np64(V)
    Uo, So, Vo = oracle.eigsvds(A, k + 1)
    r = compare_triplets(Uo[:, :k], So[:k], Vo[:, :k], Ug, Sg, Vg, So, SIG_TOL, ANG_TOL)
    say("  ->", r, "iterations", it)
    return r, it, (Ug, Sg, Vg)


def test_tall_power_law():
    A = zipf_lognormal(m=40_000, n=3_000, t=20)
    r, it, (Ug, Sg, Vg) = _check(A, 20, 12)
    assert r["ok"] and r["prefix"] >= 10, r
    assert 1 <= it < 100
    piv = np.argmax(np.abs(Vg), axis=0)
    assert np.all(Vg[piv, np.arange(Vg.shape[1])] > 0)


def test_wide_alg5_orientation():
    A = zipf_normal(m=2_500, n=30_000, t=20)
    r, it, _ = _check(A, 16, 10)
    assert r["ok"], r


def test_flat_tfidf_spectrum():
    """A few nonzeros per row with tf-idf values (the shape of the paper's Matrix 7): a flat
    spectrum, where the filter stays at low degree and the iteration needs more steps."""
    A = aminer_tfidf(m=200_000, n=8_000, t=4, seed=1008)
    r, it, _ = _check(A, 50, 28)
    assert r["ok"], r
    assert it > 2


def test_planted_closed_form():
    P = planted_blocks(m=20_000, n=4_000, blocks=80, seed=12)
    k = 30
    mat = FrPCA.from_csr(P, device=DEV)
    U, S, V, it = mat.eigsvds(k, 20, 5)
    mat.close()
    Sg = np64(S)
    sig = P.meta["sigma"][:k]
    err = float(np.max(np.abs(Sg - sig) / sig))
    say("  planted eigsvds: sigma err", err, "iterations", it)
    assert err < 1e-5


def test_iteration_limit_and_errors():
    A = zipf_lognormal(m=20_000, n=2_000, t=20)
    mat = FrPCA.from_csr(A, device=DEV)
    U, S, V, it = mat.eigsvds(10, 6, 3, tol=1e-30, max_iter=2)
    assert it == 2 and np.all(np.diff(np64(S)) <= 0)
    for args in ((0, 5, 1), (10, -1, 1), (10, 5, 0), (130, 0, 1)):
        with pytest.raises(FrpcaError) as ei:
            mat.eigsvds(args[0], args[1], 3, max_iter=args[2])
        assert ei.value.code == binding.FRPCA_EINVAL
    mat.close()
