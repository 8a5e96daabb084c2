"""The seeded synthetic workloads have the stated shapes, densities and structure."""
import numpy as np

from synth import aminer_tfidf, planted_blocks, small_decay, zipf_lognormal, zipf_normal
from synth.matrices import _ZipfSampler


def test_small_decay_shape_and_scaling():
    A = small_decay()
    A.check()
    assert (A.m, A.n) == (2000, 1000)
    assert 18_000 < A.nnz < 22_000
    norms = np.sqrt(np.bincount(np.repeat(np.arange(A.m), np.diff(A.row_ptr)),
                                weights=A.val.astype(np.float64) ** 2, minlength=A.m))
    nz = np.diff(A.row_ptr) > 0
    np.testing.assert_allclose(norms[nz] * (np.arange(A.m)[nz] + 1), 1.0, rtol=1e-6)


def test_zipf_sampler_is_exact_inverse_cdf():
    s = _ZipfSampler(50_000, 1.1)
    u = np.random.default_rng(0).random(200_000)
    ref = np.minimum(np.searchsorted(s.cdf, u, side="right"), 49_999)
    assert np.array_equal(s(u), ref)


def test_zipf_rows_distinct_and_power_law():
    A = zipf_lognormal(m=40_000, n=200_000)
    A.check()
    assert A.nnz == 40 * 40_000
    counts = np.bincount(A.col, minlength=A.n)
    assert counts[0] > 0.99 * A.m            # column 0 is in almost every row
    assert 0.45 < counts[:200].sum() / A.nnz < 0.55
    assert np.all(A.val > 0)
    B = zipf_lognormal(m=40_000, n=200_000)
    assert np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)   # seeded


def test_aminer_and_normal_variants():
    A = aminer_tfidf(m=20_000, n=323_899)
    A.check()
    assert A.nnz == 20 * 20_000 and np.all(A.val >= 0)
    Z = zipf_normal(m=10_000)
    Z.check()
    assert Z.nnz == 30 * 10_000 and abs(Z.val.mean()) < 0.05


def test_planted_blocks_exact_spectrum():
    P = planted_blocks(m=4000, n=1000, blocks=40)
    P.check()
    assert P.nnz == 4000 * 1000 // 40
    s = np.linalg.svd(P.toarray(), compute_uv=False)
    np.testing.assert_allclose(s[:40], P.meta["sigma"], rtol=1e-6)
    assert s[40] < 1e-6 * s[0]
