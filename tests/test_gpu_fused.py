"""The one-sweep pass pair (opts.fused_pass, frpca_pass(fused = 1)) against the oracle's
A^T (A Q) and against the two-product form, through the C-ABI: bit-exact on integer data
(every partial sum is an integer below 2^24, so the order of the atomic adds cannot change
it) for tall inputs with and without row-blocked columns and for wide inputs with short and
with long (power-law) segments; frpca_run with fused pass pairs against the FP64 oracle; the
options it does not combine with.
"""
import numpy as np
import pytest

import oracle
from gpu_util import ANG_TOL, SIG_TOL, compare_triplets, np64, say
from synth import Csr, random_sparse, zipf_lognormal, zipf_normal, zipf_rows

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1810_06825_amd import FrPCA, FrpcaError, binding  # noqa: E402

DEV = "cuda:0"


def _int_zipf(m, n, t, alpha, seed):
    rp, col = zipf_rows(m, n, t, alpha, seed)
    v = np.random.default_rng(seed).integers(-4, 5, size=col.size).astype(np.float32)
    v[v == 0] = 1.0
    return Csr(m, n, rp, col, v, {"workload": "integer zipf"})


def _wide_int():
    # the transpose of a tall integer Zipf matrix, as canonical CSR (power-law rows)
    import scipy.sparse as sp

    T = _int_zipf(40_000, 3_000, 12, 1.1, 43)
    W = sp.csr_matrix((T.val, T.col, T.row_ptr), shape=(T.m, T.n)).T.tocsr()
    W.sort_indices()
    return Csr(W.shape[0], W.shape[1], W.indptr.astype(np.int64), W.indices.astype(np.int32),
               W.data.astype(np.float32), {"workload": "wide integer"})


@pytest.mark.parametrize("case", ["tall_blocked", "tall_plain", "wide", "wide_heavy_columns"])
def test_pass_pair_bit_exact_on_integers(case):
    A = {"tall_blocked": lambda: _int_zipf(60_000, 3_000, 12, 1.1, 41),
         "tall_plain": lambda: random_sparse(5_000, 4_000, 0.002, seed=42, integer_values=True),
         "wide": lambda: _wide_int(),
         # power-law columns: the forward product's segments (columns) run over many windows of 64
         # entries, with odd counts in their last window
         "wide_heavy_columns": lambda: _int_zipf(3_001, 40_000, 33, 1.1, 44)}[case]()
    l = 60
    ns = min(A.m, A.n)
    X = np.random.default_rng(5).integers(-3, 4, size=(ns, l)).astype(np.float64)
    say("fused pass", case, A.m, A.n, A.nnz)
    mat = FrPCA.from_csr(A, device=DEV)
    xin = torch.zeros((ns, 64), dtype=torch.float32, device=DEV)
    xin[:, :l] = torch.from_numpy(X.astype(np.float32)).to(DEV)
    outs = []
    for fused in (0, 1):
        out = torch.full((ns, 64), 7.0, dtype=torch.float32, device=DEV)
        binding.frpca_pass(mat.h, l, xin, out, fused)
        outs.append(out.cpu().numpy())
    mat.close()
    if A.m >= A.n:
        ref = oracle.csr_tmatmul(A, oracle.csr_matmul(A, X))
    else:
        ref = oracle.csr_matmul(A, oracle.csr_tmatmul(A, X))
    assert np.abs(ref).max() < 2 ** 24
    for got in outs:
        assert np.array_equal(got[:, :l], ref)
        assert np.all(got[:, l:] == 0)


@pytest.mark.parametrize("q", [3, 4, 5])
@pytest.mark.parametrize("tall", [True, False])
def test_fused_run_matches_oracle(q, tall):
    A = zipf_lognormal(m=30_011, n=4_003, t=40) if tall else zipf_normal(m=3_001, n=20_011, t=30)
    k, s, seed = 16, 8, 91 + q
    say("fused frpca_run", A.m, A.n, f"q={q}")
    mat = FrPCA.from_csr(A, device=DEV, fused_pass=True)
    U, S, V = (np64(t) for t in mat.run(k, q, s, seed))
    mat.close()
    Uo, So, Vo, _ = oracle.frpca(A, k, q, s, seed)
    S_ritz = oracle.frpca(A, k + 1, q, s - 1, seed)[1]
    r = compare_triplets(Uo, So, Vo, U, S, V, S_ritz, SIG_TOL, ANG_TOL)
    say("  ->", r)
    assert r["ok"], r


def test_fused_option_rules():
    A = random_sparse(3_000, 500, 0.01, seed=3)
    for kw in ({"center": True}, {"panel_bf16": 1}):
        mat = FrPCA.from_csr(A, device=DEV, fused_pass=True, **kw)
        with pytest.raises(FrpcaError) as ei:
            mat.run(10, 5, 5, 1)
        assert ei.value.code == binding.FRPCA_EINVAL
        mat.close()
