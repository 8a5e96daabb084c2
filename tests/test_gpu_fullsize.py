"""Parity at the benchmark's full size: 1,000,000 x 200,000 power-law CSR (40M nonzeros), k = 100,
s = 20, q = 5, panels with leading dimension 128 (the launch configuration bench.py times).

* Omega: every entry against the oracle's Philox draw (<= 1 FP32 ulp).
* A Q and A^T Y: every output element against FP64 products of the same FP32 inputs, within the
  FP32 summation bound 4 sqrt(terms) u32 sum|terms|.
* frPCA: singular values and leading subspaces against the FP64 oracle on the same matrix and
  seed (sigma relative error <= 1e-4, sin of the largest principal angle <= 1e-3 on the block
  separated by a relative Ritz gap >= 1e-2), plus properties that hold exactly at any size:
  A V = U diag(S) (the final Rayleigh-Ritz step), orthonormal U and V, descending S, the sign
  convention, and bitwise repeatability.
"""
import numpy as np
import pytest

import oracle
from gpu_util import ANG_TOL, SIG_TOL, compare_triplets, np64, say
from synth import zipf_lognormal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1810_06825_amd import FrPCA, binding  # noqa: E402

DEV = "cuda:0"
K, S_OVER, Q_PASSES, SEED = 100, 20, 5, 20181015
L = K + S_OVER
LD = 128
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def full():
    say("full-size zipf_lognormal: generating")
    A = zipf_lognormal()
    say("full-size zipf_lognormal", A.m, A.n, A.nnz, "create")
    mat = FrPCA.from_csr(A, device=DEV)
    yield A, mat
    mat.close()


def _fp32_sum_bound(absum: np.ndarray, terms: np.ndarray) -> np.ndarray:
    return 4.0 * np.sqrt(np.maximum(terms, 1.0))[:, None] * U32 * absum + 1e-30


def test_fullsize_gaussian_and_both_products(full):
    A, mat = full
    import scipy.sparse as sp

    say("full-size Omega", A.n, L, "ld", LD)
    Om = torch.zeros((A.n, LD), dtype=torch.float32, device=DEV)
    binding.frpca_gaussian(mat.h, SEED, A.n, L, LD, Om)
    Omh = Om.cpu().numpy()
    ref = oracle.gaussian(SEED, A.n, L)
    a32 = Omh[:, :L]
    ulps = np.abs(a32.view(np.int32).astype(np.int64) - ref.astype(np.float32).view(np.int32).astype(np.int64))
    assert ulps.max() <= 1
    assert np.all(Omh[:, L:] == 0)

    say("full-size A Q", A.m, "x", LD)
    Y = torch.zeros((A.m, LD), dtype=torch.float32, device=DEV)
    binding.frpca_spmm(mat.h, 0, L, Om, 0, LD, Y, 0, LD)
    Yh = Y.cpu().numpy()
    Q64 = a32.astype(np.float64)
    exact = oracle.csr_matmul(A, Q64)
    absA = sp.csr_matrix((np.abs(A.val.astype(np.float64)), A.col, A.row_ptr), shape=(A.m, A.n))
    bound = _fp32_sum_bound(absA @ np.abs(Q64), np.diff(A.row_ptr).astype(np.float64))
    err = np.abs(Yh[:, :L] - exact)
    say("  A Q max err / bound", float((err / bound).max()))
    assert np.all(err <= bound)
    assert np.all(Yh[:, L:] == 0)

    say("full-size A^T Y", A.n, "x", LD)
    X = torch.zeros((A.n, LD), dtype=torch.float32, device=DEV)
    binding.frpca_spmm(mat.h, 1, L, Y, 0, LD, X, 0, LD)
    Xh = X.cpu().numpy()
    Y64 = Yh[:, :L].astype(np.float64)
    exact = oracle.csr_tmatmul(A, Y64)
    colcnt = np.bincount(A.col, minlength=A.n).astype(np.float64)
    bound = _fp32_sum_bound(absA.T @ np.abs(Y64), colcnt)
    err = np.abs(Xh[:, :L] - exact)
    say("  A^T Y max err / bound", float((err / bound).max()), "hottest column count", int(colcnt.max()))
    assert np.all(err <= bound)
    assert np.all(Xh[:, L:] == 0)


def _run(mat, A):
    U = torch.empty((A.m, K), dtype=torch.float32, device=DEV)
    S = torch.empty((K,), dtype=torch.float32, device=DEV)
    V = torch.empty((A.n, K), dtype=torch.float32, device=DEV)
    mat.run(K, Q_PASSES, S_OVER, SEED, out=(U, S, V))
    torch.cuda.synchronize()
    return U, S, V


def test_fullsize_frpca_matches_oracle(full):
    A, mat = full
    say("full-size frpca_run", f"k={K} q={Q_PASSES} s={S_OVER}")
    U, S, V = _run(mat, A)
    Ug, Sg, Vg = np64(U), np64(S), np64(V)
    # one oracle run with k+1 (same l, so the same sketch and Ritz values) gives both the
    # reference triplets and the Ritz value past k for the gap test
    say("full-size oracle (FP64, CPU)")
    Uo, So, Vo, _ = oracle.frpca(A, K + 1, Q_PASSES, S_OVER - 1, SEED)
    r = compare_triplets(Uo[:, :K], So[:K], Vo[:, :K], Ug, Sg, Vg, So, SIG_TOL, ANG_TOL)
    say("  ->", r)
    assert r["ok"], r
    assert r["prefix"] >= 10


def test_fullsize_properties(full):
    A, mat = full
    say("full-size frpca_run properties")
    U, S, V = _run(mat, A)
    U2, S2, V2 = _run(mat, A)
    assert torch.equal(U, U2) and torch.equal(S, S2) and torch.equal(V, V2)
    Sg = np64(S)
    assert np.all(Sg > 0) and np.all(np.diff(Sg) <= 0)
    Ud, Vd = U.double(), V.double()
    eye = torch.eye(K, dtype=torch.float64, device=DEV)
    ou = float((Ud.T @ Ud - eye).abs().max())
    ov = float((Vd.T @ Vd - eye).abs().max())
    say("  orthonormality U, V", ou, ov)
    assert ou <= 1e-5 and ov <= 1e-5
    Vg, Ug = np64(V), np64(U)
    AV = oracle.csr_matmul(A, Vg)
    rr = float(np.abs(AV - Ug * Sg).max() / Sg[0])
    say("  max |A V - U S| / sigma_1", rr)
    assert rr <= 1e-5
    piv = np.argmax(np.abs(Vg), axis=0)
    assert np.all(Vg[piv, np.arange(K)] > 0)
