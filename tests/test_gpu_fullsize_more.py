"""Parity at full size for the two other large workloads, in the launch configuration of
bench.py (panels with leading dimension 128, k = 100, s = 20):

* aminer_tfidf, 12,869,521 x 323,899 (257,390,420 nnz, Zipf 1.0 columns, tf-idf values),
  q = 5: sampled rows of A Q and sampled columns of A^T Y (the hottest column, about
  10M terms, among them) against FP64 sums of the same FP32 inputs, on 128- and 64-column
  panels; sampled rows of
  A V = U diag(S) in FP64; and the whole method at q = 3, 5 and 7 against the oracle on the
  whole matrix. Properties that hold at any size: orthonormal U and V, descending S, the sign
  convention, repeatability.
* zipf_normal, 500,000 x 100,000 (15,000,000 nnz, the differentiated workload), k = 50,
  s = 10, q = 4: the forward against the FP64 oracle on the whole matrix, and the gradient of
  sum(sigma) + ||U W||^2 (whose second term is invariant) against its closed form
  sum_i u_i[r] v_i[c] at every nonzero.
* planted_blocks, 200,000 x 50,000 (50,000,000 nnz, exact sigma_i = 10^(-3 i / 200)),
  q = 3 and 5 against the FP64 oracle on the whole matrix (about a minute of CPU each), the
  leading values against the closed form, q = 1 rejected, q = 2 and 7 by their properties.
"""
import time

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from gpu_util import ANG_TOL, SIG_TOL, compare_triplets, np64, say
from synth import Csr, aminer_tfidf, planted_blocks, zipf_normal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1810_06825_amd import FrPCA, FrpcaError, binding, frpca_autograd  # noqa: E402

DEV = "cuda:0"
K, S_OVER, SEED = 100, 20, 20181015
L = K + S_OVER
LD = 128
U32 = 2.0 ** -24


def _sum_bound(absum, terms):
    return 4.0 * np.sqrt(np.maximum(terms, 1.0))[:, None] * U32 * absum + 1e-30


def _run(mat, A, q):
    U = torch.empty((A.m, K), dtype=torch.float32, device=DEV)
    S = torch.empty((K,), dtype=torch.float32, device=DEV)
    V = torch.empty((A.n, K), dtype=torch.float32, device=DEV)
    mat.run(K, q, S_OVER, SEED, out=(U, S, V))
    torch.cuda.synchronize()
    return U, S, V


def _gram_identity_err(X):
    # max |X^T X - I| in FP64 on the GPU, in row chunks (X is m x k FP32)
    G = torch.zeros((K, K), dtype=torch.float64, device=DEV)
    for r0 in range(0, X.shape[0], 1 << 22):
        c = X[r0:r0 + (1 << 22)].double()
        G += c.T @ c
    return float((G - torch.eye(K, dtype=torch.float64, device=DEV)).abs().max())


@pytest.fixture(scope="module")
def aminer():
    say("full-size aminer_tfidf: generating")
    A = aminer_tfidf()
    say("full-size aminer_tfidf", A.m, A.n, A.nnz, "create")
    mat = FrPCA.from_csr(A, device=DEV)
    yield A, mat
    mat.close()


@pytest.mark.parametrize("L,LD", [(L, LD), (60, 64)])
def test_aminer_products_sampled(aminer, L, LD):
    # 64-column panels run the four-nonzeros-per-gather kernels in all three modes: the
    # forward product, the row-blocked hot part (sweep) and the tail part, whose 3.3 GB
    # gathered panel takes streaming loads
    A, mat = aminer
    rng = np.random.default_rng(11)
    Acsr = sp.csr_matrix((A.val.astype(np.float64), A.col, A.row_ptr), shape=(A.m, A.n))
    say("aminer Omega + A Q", A.n, L, LD)
    Om = torch.zeros((A.n, LD), dtype=torch.float32, device=DEV)
    binding.frpca_gaussian(mat.h, SEED, A.n, L, LD, Om)
    Q64 = Om[:, :L].double().cpu().numpy()
    Y = torch.zeros((A.m, LD), dtype=torch.float32, device=DEV)
    binding.frpca_spmm(mat.h, 0, L, Om, 0, LD, Y, 0, LD)
    nnz_row = np.diff(A.row_ptr)
    rows = np.unique(np.concatenate([rng.choice(A.m, 20_000, replace=False), np.argsort(nnz_row)[-64:],
                                     [0, A.m - 1]]))
    rows_t = torch.from_numpy(rows).to(DEV)
    Yr = Y.index_select(0, rows_t).cpu().numpy()
    Ar = Acsr[rows]
    exact = Ar @ Q64
    bound = _sum_bound(abs(Ar) @ np.abs(Q64), nnz_row[rows].astype(np.float64))
    err = np.abs(Yr[:, :L] - exact)
    say("  A Q sampled rows: max err / bound", float((err / bound).max()))
    assert np.all(err <= bound)
    assert np.all(Yr[:, L:] == 0)

    say("aminer A^T Y")
    X = torch.zeros((A.n, LD), dtype=torch.float32, device=DEV)
    binding.frpca_spmm(mat.h, 1, L, Y, 0, LD, X, 0, LD)
    colcnt = np.bincount(A.col, minlength=A.n)
    cols = np.unique(np.concatenate([rng.choice(A.n, 2_000, replace=False), np.argsort(colcnt)[-16:],
                                     [0, A.n - 1]]))
    AT = Acsr.T.tocsr()[cols]                      # the sampled columns of A as rows
    need = np.unique(AT.indices)                   # rows of Y those columns touch
    Yn = Y.index_select(0, torch.from_numpy(need).to(DEV))[:, :L].double().cpu().numpy()
    ATn = sp.csr_matrix((AT.data, np.searchsorted(need, AT.indices), AT.indptr), shape=(len(cols), len(need)))
    exact = ATn @ Yn
    bound = _sum_bound(abs(ATn) @ np.abs(Yn), colcnt[cols].astype(np.float64))
    Xc = X.index_select(0, torch.from_numpy(cols).to(DEV)).cpu().numpy()
    err = np.abs(Xc[:, :L] - exact)
    say("  A^T Y sampled columns: max err / bound", float((err / bound).max()), "hottest column", int(colcnt.max()))
    assert np.all(err <= bound)
    assert np.all(Xc[:, L:] == 0)


def test_aminer_frpca_properties(aminer):
    A, mat = aminer
    say("aminer frpca_run q=5 properties")
    U, S, V = _run(mat, A, 5)
    U2, S2, V2 = _run(mat, A, 5)
    assert torch.equal(U, U2) and torch.equal(S, S2) and torch.equal(V, V2)
    Sg = np64(S)
    assert np.all(Sg > 0) and np.all(np.diff(Sg) <= 0)
    ou, ov = _gram_identity_err(U), _gram_identity_err(V)
    say("  orthonormality U, V", ou, ov)
    assert ou <= 1e-5 and ov <= 1e-5
    Vg = np64(V)
    piv = np.argmax(np.abs(Vg), axis=0)
    assert np.all(Vg[piv, np.arange(K)] > 0)
    # the final Rayleigh-Ritz step: A V = U diag(S), on sampled rows in FP64
    rows = np.unique(np.random.default_rng(12).choice(A.m, 50_000, replace=False))
    Acsr = sp.csr_matrix((A.val.astype(np.float64), A.col, A.row_ptr), shape=(A.m, A.n))
    AV = Acsr[rows] @ Vg
    Ur = U.index_select(0, torch.from_numpy(rows).to(DEV)).double().cpu().numpy()
    rr = float(np.abs(AV - Ur * Sg).max() / Sg[0])
    say("  sampled max |A V - U S| / sigma_1", rr)
    assert rr <= 1e-5


@pytest.mark.timeout(1200)
def test_aminer_whole_matrix_matches_oracle(aminer):
    """The benchmark's job itself: q = 5 on the whole 12.9M x 324K matrix against the FP64
    oracle on the same matrix (about two minutes of host CPU and 60 GB of host memory)."""
    A, mat = aminer
    say("aminer frpca_run q=5 on the GPU")
    U, S, V = _run(mat, A, 5)
    Sg, Vg = np64(S), np64(V)
    Ug = np64(U)
    del U, S, V
    t0 = time.time()
    Uo, So, Vo, _ = oracle.frpca(A, K + 1, 5, S_OVER - 1, SEED,
                                 log=lambda msg: say(f"  oracle {msg} ({time.time() - t0:.0f} s)"))
    say("  oracle on the whole matrix took", round(time.time() - t0, 1), "s")
    r = compare_triplets(Uo[:, :K], So[:K], Vo[:, :K], Ug, Sg, Vg, So, SIG_TOL, ANG_TOL)
    say("  ->", r)
    assert r["ok"], r
    assert r["prefix"] >= 10


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("q", [3, 7])
def test_aminer_other_pass_counts(aminer, q):
    """q = 3 and 7 on the whole 12.9M x 324K matrix: orthonormal factors, descending values,
    and the whole method against the FP64 oracle on the same matrix (one and three power
    steps; about one and two minutes of host CPU)."""
    A, mat = aminer
    say(f"aminer frpca_run q={q}")
    U, S, V = _run(mat, A, q)
    Sg, Ug, Vg = np64(S), np64(U), np64(V)
    assert np.all(Sg > 0) and np.all(np.diff(Sg) <= 0)
    ou, ov = _gram_identity_err(U), _gram_identity_err(V)
    say("  orthonormality U, V", ou, ov)
    assert ou <= 1e-5 and ov <= 1e-5
    del U, S, V
    t0 = time.time()
    Uo, So, Vo, _ = oracle.frpca(A, K + 1, q, S_OVER - 1, SEED,
                                 log=lambda msg: say(f"  oracle {msg} ({time.time() - t0:.0f} s)"))
    r = compare_triplets(Uo[:, :K], So[:K], Vo[:, :K], Ug, Sg, Vg, So, SIG_TOL, ANG_TOL)
    say(f"  q={q} vs oracle ->", r)
    assert r["ok"], r


def test_differentiated_workload_full_size():
    A = zipf_normal()
    k, q, s = 50, 4, 10
    say("full-size zipf_normal", A.m, A.n, A.nnz, f"k={k} q={q} s={s}")
    mat = FrPCA.from_csr(A, device=DEV)
    vals = torch.from_numpy(A.val).to(DEV).requires_grad_(True)
    U, S, V = frpca_autograd(vals, mat, k, q, s, SEED)
    W = torch.from_numpy(np.random.default_rng(7).standard_normal((k, 8)).astype(np.float32)).to(DEV)
    loss = S.sum() + ((U @ W) ** 2).sum()
    loss.backward()
    Ug, Sg, Vg = np64(U), np64(S), np64(V)
    g = np64(vals.grad)
    mat.close()
    say("  oracle (FP64, CPU)")
    Uo, So, Vo, _ = oracle.frpca(A, k + 1, q, s - 1, SEED)
    r = compare_triplets(Uo[:, :k], So[:k], Vo[:, :k], Ug, Sg, Vg, So, SIG_TOL, ANG_TOL)
    say("  forward ->", r)
    assert r["ok"], r
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    ref = np.empty(A.nnz)
    for e0 in range(0, A.nnz, 1 << 21):
        e1 = min(A.nnz, e0 + (1 << 21))
        ref[e0:e1] = np.einsum("ij,ij->i", Ug[rows[e0:e1]], Vg[A.col[e0:e1]])
    err = float(np.abs(g - ref).max() / np.abs(ref).max())
    say("  gradient vs sum_i u_i[r] v_i[c]: rel err", err)
    assert err < 1e-4


_ORACLE = {}


def _oracle_planted(P, q):
    # one FP64 run with k + 1 per pass count (same l, so the same sketch), shared by the tests
    if q not in _ORACLE:
        say("  planted oracle (FP64, CPU)", f"q={q}")
        _ORACLE[q] = oracle.frpca(P, K + 1, q, S_OVER - 1, SEED)
    return _ORACLE[q]


@pytest.fixture(scope="module")
def planted():
    say("full-size planted_blocks: generating")
    P = planted_blocks()
    say("full-size planted_blocks", P.m, P.n, P.nnz)
    mat = FrPCA.from_csr(P, device=DEV)
    yield P, mat
    mat.close()


@pytest.mark.parametrize("q", [3, 5])
def test_planted_matches_oracle_and_closed_form(planted, q):
    P, mat = planted
    say("planted frpca_run", f"q={q}")
    U, S, V = _run(mat, P, q)
    Ug, Sg, Vg = np64(U), np64(S), np64(V)
    Uo, So, Vo, _ = _oracle_planted(P, q)
    r = compare_triplets(Uo[:, :K], So[:K], Vo[:, :K], Ug, Sg, Vg, So, SIG_TOL, ANG_TOL)
    sig = P.meta["sigma"][:K]
    lead = float(np.max(np.abs(Sg[:10] - sig[:10]) / sig[:10]))
    say("  ->", r, "| leading 10 vs closed form", lead)
    assert r["ok"], r
    # Rayleigh-Ritz values never exceed the true ones (FP32 slack)
    assert np.all(Sg <= sig * (1 + 1e-5))
    if q == 5:
        # two power steps: sigma_10 converges by (sigma_121 / sigma_10)^4 ~ 2e-7
        assert lead < 1e-4


def test_planted_pass_counts(planted):
    """q = 1 is rejected; q = 2 and 7 give orthonormal factors whose values interlace the
    planted ones and, at q = 7, match the leading ones."""
    P, mat = planted
    say("planted q=1 rejected, q=2 and 7 properties")
    with pytest.raises(FrpcaError) as ei:
        _run(mat, P, 1)
    assert ei.value.code == binding.FRPCA_EINVAL
    sig = P.meta["sigma"][:K]
    for q in (2, 7):
        U, S, V = _run(mat, P, q)
        Sg = np64(S)
        ou, ov = _gram_identity_err(U), _gram_identity_err(V)
        lead = float(np.max(np.abs(Sg[:10] - sig[:10]) / sig[:10]))
        say(f"  q={q}: orthonormality", ou, ov, "leading 10 vs closed form", lead)
        assert ou <= 1e-5 and ov <= 1e-5
        assert np.all(np.diff(Sg) <= 0) and np.all(Sg <= sig * (1 + 1e-5))
        if q == 7:
            assert lead < 1e-5


def test_planted_precision_variants_stated(planted):
    """BF16 panels and the FP32-MFMA Gram next to the default, against the FP64 oracle."""
    P, _ = planted
    Uo, So, Vo, _ = _oracle_planted(P, 5)
    for kw in ({"panel_bf16": True}, {"gram_f32": True}):
        m2 = FrPCA.from_csr(P, device=DEV, **kw)
        U, S, V = _run(m2, P, 5)
        m2.close()
        r = compare_triplets(Uo[:, :K], So[:K], Vo[:, :K], np64(U), np64(S), np64(V), So, 1.0, 1.0)
        say("  planted q=5", kw, "->", r)
        assert r["sig_err"] < 1e-2
