"""Step-level parity of the HIP kernels against the FP64 oracle, through the C-ABI.

Each test names its case before launching; sizes span several tiles / merge partitions and
end on ragged tails.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
from gpu_util import fp32_ulp_diff, np64, say, sin_theta
from synth import random_sparse, zipf_lognormal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1810_06825_amd import FrPCA, binding  # noqa: E402

DEV = "cuda:0"


def _mat(A, **kw):
    return FrPCA.from_csr(A, device=DEV, **kw)


def test_gaussian_matches_philox_reference():
    for seed, rows, l, ld in ((20181015, 1000, 15, 32), (7, 777, 120, 128), (2**40 + 3, 33, 1, 2)):
        say("gaussian", seed, rows, l, ld)
        A = random_sparse(8, 8, 0.5, seed=1)
        mat = _mat(A)
        out = torch.full((rows, ld), 7.0, dtype=torch.float32, device=DEV)
        binding.frpca_gaussian(mat.h, seed, rows, l, ld, out)
        g = out.cpu().numpy()
        ref = oracle.gaussian(seed, rows, l).astype(np.float32)
        ulp = fp32_ulp_diff(g[:, :l], ref)
        assert ulp.max() <= 1 and (ulp == 0).mean() > 0.999
        assert np.all(g[:, l:] == 0.0)


@pytest.mark.parametrize("case", ["random", "zipf", "empty"])
def test_csc_mirror_bit_exact(case):
    if case == "random":
        A = random_sparse(3001, 1999, 0.004, seed=5, empty_rows=(0, 17, 3000), empty_cols=(0, 1, 1998))
    elif case == "zipf":
        A = zipf_lognormal(m=50_000, n=20_000, t=40)
    else:
        A = random_sparse(50, 40, 0.0, seed=1)
    say("csc mirror", case, A.m, A.n, A.nnz)
    mat = _mat(A)
    cp = torch.empty(A.n + 1, dtype=torch.int64, device=DEV)
    row = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=DEV)
    perm = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=DEV)
    binding.frpca_export_csc(mat.h, cp, row, perm)
    col_ptr, row_o, perm_o = oracle.csc_mirror(A)
    assert np.array_equal(cp.cpu().numpy(), col_ptr)
    assert np.array_equal(row.cpu().numpy()[:A.nnz], row_o)
    assert np.array_equal(perm.cpu().numpy()[:A.nnz], perm_o)


def _spmm(mat, trans, X, ld, in_bf16=False, out_bf16=False):
    rows_out = mat.n if trans else mat.m
    l = X.shape[1]
    xin = torch.zeros((X.shape[0], ld), dtype=torch.float32)
    xin[:, :l] = torch.from_numpy(X.astype(np.float32))
    if in_bf16:
        xin = xin.to(torch.bfloat16).view(torch.int16)
    xin = xin.to(DEV)
    if out_bf16:
        out = torch.full((rows_out, ld), 3, dtype=torch.int16, device=DEV)
    else:
        out = torch.full((rows_out, ld), 3.0, dtype=torch.float32, device=DEV)
    binding.frpca_spmm(mat.h, trans, l, xin, int(in_bf16), ld, out, int(out_bf16), ld)
    if out_bf16:
        out = out.view(torch.bfloat16)
    return out.float().cpu().numpy()


@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("ld", [64, 128])
def test_spmm_integer_values_bit_exact(trans, ld):
    # ld 64: one column half; ld 128: the halves on separate XCD groups
    A = random_sparse(2500, 1700, 0.01, seed=11, empty_rows=(3, 2499), empty_cols=(0, 5), integer_values=True)
    rows_in = A.m if trans else A.n
    l = ld - 4
    X = np.random.default_rng(2).integers(-8, 9, size=(rows_in, l)).astype(np.float64)
    say("spmm integer", trans, ld, A.m, A.n, A.nnz)
    mat = _mat(A)
    got = _spmm(mat, trans, X, ld)
    ref = oracle.csr_tmatmul(A, X) if trans else oracle.csr_matmul(A, X)
    assert np.array_equal(got[:, :l], ref)
    assert np.all(got[:, l:] == 0)


@pytest.mark.parametrize("trans", [0, 1])
@pytest.mark.parametrize("l", [15, 120])
def test_spmm_float_parity_power_law(trans, l):
    # heavy Zipf columns: column 0 holds ~every row, so the transposed product's segments
    # span hundreds of merge partitions and exercise the carry fix-up
    A = zipf_lognormal(m=60_001, n=9_999, t=40)
    rows_in = A.m if trans else A.n
    X = np.random.default_rng(3).standard_normal((rows_in, l))
    say("spmm float", trans, l, A.m, A.n, A.nnz)
    mat = _mat(A)
    ld = (l + 31) // 32 * 32
    got = _spmm(mat, trans, X, ld)[:, :l]
    Xf = X.astype(np.float32).astype(np.float64)
    ref = oracle.csr_tmatmul(A, Xf) if trans else oracle.csr_matmul(A, Xf)
    absA = A.to_scipy()
    absA.data = np.abs(absA.data)
    bound = (absA.T if trans else absA) @ np.abs(Xf)
    # FP32 accumulation in merge-path partitions plus their carries: well inside ~170 ulp
    # of the absolute sum; an indexing mistake would be O(1) relative
    assert np.all(np.abs(got - ref) <= 1e-5 * bound + 1e-30)


@pytest.mark.parametrize("trans", [0, 1])
def test_spmm_width_not_multiple_of_4(trans):
    # 14 computed columns: the two-column-per-lane kernel instead of the paired 16-byte one
    A = zipf_lognormal(m=30_011, n=4_003, t=20)
    rows_in = A.m if trans else A.n
    X = np.random.default_rng(5).standard_normal((rows_in, 13))
    say("spmm width 14", trans, A.m, A.n, A.nnz)
    mat = _mat(A)
    got = _spmm(mat, trans, X, 14)[:, :13]
    Xf = X.astype(np.float32).astype(np.float64)
    ref = oracle.csr_tmatmul(A, Xf) if trans else oracle.csr_matmul(A, Xf)
    absA = A.to_scipy()
    absA.data = np.abs(absA.data)
    bound = (absA.T if trans else absA) @ np.abs(Xf)
    assert np.all(np.abs(got - ref) <= 1e-5 * bound + 1e-30)


@pytest.mark.parametrize("layout", ["all_hot", "no_hot", "mixed", "tiny_hot"])
def test_transpose_product_layouts(layout):
    """A^T Y through the row-blocked order when every column is frequent (no tail part), when
    none is (plain column order), for a mix over several row blocks, and for a hot part of a
    dozen partitions (a sweep grid of fewer blocks than XCDs); exact on integers."""
    if layout == "tiny_hot":
        A = random_sparse(300, 4, 0.9, seed=24, integer_values=True)
    elif layout == "all_hot":
        A = random_sparse(3000, 50, 0.3, seed=21, integer_values=True)
    elif layout == "no_hot":
        A = random_sparse(20_000, 20_000, 1e-4, seed=22, integer_values=True)
    else:
        A = random_sparse(30_000, 700, 0.02, seed=23, empty_cols=(3, 699), integer_values=True)
    Y = np.random.default_rng(6).integers(-8, 9, size=(A.m, 60)).astype(np.float64)
    say("transpose layout", layout, A.m, A.n, A.nnz)
    mat = _mat(A)
    info = mat.info()
    if layout in ("all_hot", "tiny_hot"):
        assert info["hot_cols"] == A.n and info["hot_nnz"] == A.nnz
    elif layout == "no_hot":
        assert info["hot_cols"] == 0
    else:
        assert 0 < info["hot_cols"] < A.n and info["row_blocks"] == 8
    got = _spmm(mat, 1, Y, 64)
    assert np.array_equal(got[:, :60], oracle.csr_tmatmul(A, Y))
    assert np.all(got[:, 60:] == 0)


@pytest.mark.parametrize("trans", [0, 1])
def test_spmm_bf16_panels(trans):
    A = random_sparse(4000, 3000, 0.01, seed=12)
    rows_in = A.m if trans else A.n
    X = np.random.default_rng(4).standard_normal((rows_in, 120))
    say("spmm bf16", trans)
    mat = _mat(A)
    got = _spmm(mat, trans, X, 128, in_bf16=True, out_bf16=True)[:, :120]
    xb = torch.from_numpy(X.astype(np.float32)).to(torch.bfloat16).double().numpy()
    ref = oracle.csr_tmatmul(A, xb) if trans else oracle.csr_matmul(A, xb)
    # output rounded to bf16 (relative 2^-9) on top of FP32 accumulation
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("l", [1, 15, 40, 60, 100, 120, 128])
def test_gram_fp64_accumulation(l):
    rows = 50_003
    X = np.random.default_rng(l).standard_normal((rows, l)).astype(np.float32)
    ld = max(l, 4)
    say("gram", rows, l)
    mat = _mat(random_sparse(8, 8, 0.5, seed=1))
    Xd = torch.zeros((rows, ld), dtype=torch.float32)
    Xd[:, :l] = torch.from_numpy(X)
    Xd = Xd.to(DEV)
    G = torch.zeros((l, l), dtype=torch.float64, device=DEV)
    binding.frpca_gram(mat.h, rows, l, Xd, ld, G)
    ref = X.astype(np.float64).T @ X.astype(np.float64)
    Gg = G.cpu().numpy()
    assert np.abs(Gg - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(Gg, Gg.T)


@pytest.mark.parametrize("f32", [False, True])
def test_gram_padded_panel_padding_not_used(f32):
    """Panels padded to a multiple of 32 columns take the unmasked-load path: the padding
    (here NaN) may enter only Gram entries outside l x l, which are dropped. Rows cover full
    8-row stretches in all blocks but the last, which keeps the masked path."""
    rows, l, ld = 100_001, 120, 128
    X = np.random.default_rng(31).standard_normal((rows, l)).astype(np.float32)
    say("gram padded NaN", rows, l, ld, "f32" if f32 else "f64")
    mat = _mat(random_sparse(8, 8, 0.5, seed=1), gram_f32=f32)
    Xd = torch.full((rows, ld), float("nan"), dtype=torch.float32)
    Xd[:, :l] = torch.from_numpy(X)
    Xd = Xd.to(DEV)
    G = torch.zeros((l, l), dtype=torch.float64, device=DEV)
    binding.frpca_gram(mat.h, rows, l, Xd, ld, G)
    X64 = X.astype(np.float64)
    ref = X64.T @ X64
    Gg = G.cpu().numpy()
    assert np.all(np.isfinite(Gg))
    bound = (32 * 2.0 ** -24 if f32 else 1e-13) * (np.abs(X64).T @ np.abs(X64)) + 1e-13 * np.abs(ref).max()
    assert np.all(np.abs(Gg - ref) <= bound)


@pytest.mark.parametrize("l", [1, 15, 40, 60, 100, 128])
def test_gram_fp32_mfma_variant(l):
    """FP32 matrix-core Gram (opts.gram_f32): every FP32 partial sums 16 rows, so each entry is
    within gamma_16 (here 2 * 16 u32, one rounding per product and per addition) of
    sum_r |x_ri| |x_rj| of the exact FP64 value; a sum running longer in FP32, or a misplaced
    output entry, breaks that bound."""
    rows = 50_003
    X = np.random.default_rng(100 + l).standard_normal((rows, l)).astype(np.float32)
    ld = max(l, 4)
    say("gram fp32 mfma", rows, l)
    mat = _mat(random_sparse(8, 8, 0.5, seed=1), gram_f32=True)
    Xd = torch.zeros((rows, ld), dtype=torch.float32)
    Xd[:, :l] = torch.from_numpy(X)
    Xd = Xd.to(DEV)
    G = torch.zeros((l, l), dtype=torch.float64, device=DEV)
    binding.frpca_gram(mat.h, rows, l, Xd, ld, G)
    X64 = X.astype(np.float64)
    ref = X64.T @ X64
    absref = np.abs(X64).T @ np.abs(X64)
    Gg = G.cpu().numpy()
    err = np.abs(Gg - ref)
    assert np.all(err <= 32 * 2.0 ** -24 * absref + 1e-13 * np.abs(ref).max())
    assert np.array_equal(Gg, Gg.T)
    # the FP32 sums did run: the FP64 path is exact to about 1e-15 relative
    assert err.max() > 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("l,kind", [(15, "spread"), (60, "spread"), (120, "spread"), (128, "cluster"),
                                    (7, "degenerate"), (2, "spread"), (1, "spread"), (3, "spread"),
                                    (128, "indefinite"), (100, "multiplicity"), (100, "psd_wide"),
                                    (64, "identity"), (20, "diagonal"), (120, "gram_rank40")])
def test_eig(l, kind):
    """Eigendecomposition of symmetric matrices with wide, clustered, repeated, indefinite and
    rank-deficient spectra: eigenvalues, residual and orthogonality at FP64 level."""
    rng = np.random.default_rng(l)
    Qr = np.linalg.qr(rng.standard_normal((l, l)))[0]
    spectra = {
        "spread": lambda: np.geomspace(1e-8, 1e4, l),
        "cluster": lambda: np.concatenate([[1e3, 1e2, 10, 1e-3, 1e-6], 1.0 + 1e-9 * rng.standard_normal(l - 5)]),
        "degenerate": lambda: np.array([0.0, 0.0, 1.0, 1.0, 1.0, 5.0, 9.0]),
        "multiplicity": lambda: np.repeat([1.0, 2.0, 3.0, 4.0], l // 4),
        "psd_wide": lambda: np.concatenate([np.geomspace(1, 1e-14, l // 2), np.zeros(l - l // 2)]),
    }
    if kind in spectra:
        G = (Qr * spectra[kind]()) @ Qr.T
    elif kind == "indefinite":
        B = rng.standard_normal((l, l))
        G = B + B.T
    elif kind == "identity":
        G = np.eye(l)
    elif kind == "diagonal":
        G = np.diag(rng.permutation(np.arange(1.0, l + 1)))
    else:  # gram_rank40
        X = rng.standard_normal((500, 40)) @ rng.standard_normal((40, l))
        G = X.T @ X
    G = (G + G.T) / 2
    say("eig", l, kind)
    mat = _mat(random_sparse(8, 8, 0.5, seed=1))
    Gd = torch.from_numpy(G).to(DEV)
    W = torch.zeros((l, l), dtype=torch.float64, device=DEV)
    dd = torch.zeros(l, dtype=torch.float64, device=DEV)
    binding.frpca_eig(mat.h, l, Gd, W, dd)
    Wg, dg = W.cpu().numpy(), dd.cpu().numpy()
    dref = np.linalg.eigvalsh(G)
    nrm = np.abs(dref).max()
    assert np.all(np.diff(dg) >= 0)
    assert np.abs(dg - dref).max() <= 1e-12 * nrm
    assert np.abs(G @ Wg - Wg * dg).max() <= 1e-12 * nrm
    assert np.abs(Wg.T @ Wg - np.eye(l)).max() <= 1e-12


def test_eigsvd_step_matches_oracle():
    rows, l = 20_001, 40
    X = (np.random.default_rng(9).standard_normal((rows, l)) * np.geomspace(1, 100, l)).astype(np.float32)
    say("eigsvd", rows, l)
    mat = _mat(random_sparse(8, 8, 0.5, seed=1))
    Xd = torch.from_numpy(X).to(DEV)
    Q = torch.zeros((rows, l), dtype=torch.float32, device=DEV)
    S = torch.zeros(l, dtype=torch.float64, device=DEV)
    binding.frpca_eigsvd(mat.h, rows, l, Xd, l, Q, l, S, 0.0)
    Uo, So, Vo, _ = oracle.eigsvd(X.astype(np.float64))
    np.testing.assert_allclose(S.cpu().numpy(), So, rtol=1e-10)
    Qg = np64(Q)
    for j in range(l):  # ascending columns, each equal up to sign
        c = abs(Qg[:, j] @ Uo[:, j])
        assert abs(c - 1) < 1e-5
    assert np.abs(Qg.T @ Qg - np.eye(l)).max() < 1e-5


@pytest.mark.parametrize("l", [15, 60, 120])
def test_lu_basis(l):
    rows = 30_011
    X = np.random.default_rng(l + 1).standard_normal((rows, l)).astype(np.float32)
    ld = (l + 31) // 32 * 32
    say("lu", rows, l)
    mat = _mat(random_sparse(8, 8, 0.5, seed=1))
    Xd = torch.zeros((rows, ld), dtype=torch.float32)
    Xd[:, :l] = torch.from_numpy(X)
    Xd = Xd.to(DEV)
    Q = torch.zeros((rows, l), dtype=torch.float32, device=DEV)
    nd = binding.frpca_lu(mat.h, rows, l, Xd, ld, Q, l, 0.0)
    assert nd == 0
    Qg = np64(Q)
    # Lemma 3: P^T L spans range(X)
    assert sin_theta(X.astype(np.float64), Qg) < 1e-5
    # the oracle's partial-pivoting basis spans the same space
    Lo = oracle.lu_pl(X.astype(np.float64))[0]
    assert sin_theta(Lo, Qg) < 1e-5
    # pivot rows form a unit lower-triangular block; entries stay bounded
    piv = [int(np.argmax(np.abs(Qg[:, j] - 1.0) < 1e-6)) for j in range(l)]
    blk = Qg[piv]
    assert np.allclose(np.diag(blk), 1.0, atol=1e-6)
    assert np.abs(np.triu(blk, 1)).max() < 1e-6
    assert np.abs(Qg).max() < 4.0


def test_lu_rank_deficient_drops_zero_columns():
    rows, l = 5000, 12
    rng = np.random.default_rng(3)
    X = np.zeros((rows, 32), np.float32)
    X[:, :l] = rng.standard_normal((rows, 6)) @ rng.standard_normal((6, l))
    X[:, 3] = 0.0  # an exactly-zero column has no pivot at any node
    say("lu rank-deficient")
    mat = _mat(random_sparse(8, 8, 0.5, seed=1))
    Q = torch.zeros((rows, l), dtype=torch.float32, device=DEV)
    nd = binding.frpca_lu(mat.h, rows, l, torch.from_numpy(X).to(DEV), 32, Q, l, 1e-4)
    Qg = np64(Q)
    # rank 6: the root drops the 6 columns whose best pivot is FP32 noise, plus none more
    assert nd == 6 and np.all(Qg[:, 3] == 0)
    kept = [j for j in range(l) if np.abs(Qg[:, j]).max() > 0]
    assert len(kept) == 6
    Ux = np.linalg.svd(X[:, :l].astype(np.float64), full_matrices=False)[0][:, :6]
    assert sin_theta(Ux, Qg[:, kept]) < 1e-4 and sin_theta(Qg[:, kept], Ux) < 1e-4


def test_tsmm_fp64_accumulation():
    rows, kd, c = 100_003, 120, 100
    X = np.random.default_rng(5).standard_normal((rows, kd)).astype(np.float32)
    B = np.random.default_rng(6).standard_normal((kd, c))
    say("tsmm", rows, kd, c)
    mat = _mat(random_sparse(8, 8, 0.5, seed=1))
    out = torch.zeros((rows, c), dtype=torch.float32, device=DEV)
    binding.frpca_tsmm(mat.h, rows, kd, c, torch.from_numpy(X).to(DEV), kd, torch.from_numpy(B).to(DEV), out, c)
    ref = X.astype(np.float64) @ B
    assert np.all(np.abs(np64(out) - ref) <= 6e-8 * np.abs(ref) + 1e-12 * np.abs(X) @ np.abs(B))


def test_sddmm_matches_row_dots():
    A = zipf_lognormal(m=20_000, n=5_000, t=40)
    w = 50
    rng = np.random.default_rng(8)
    P1, P2 = rng.standard_normal((A.m, w)).astype(np.float32), rng.standard_normal((A.m, w)).astype(np.float32)
    Q1, Q2 = rng.standard_normal((A.n, w)).astype(np.float32), rng.standard_normal((A.n, w)).astype(np.float32)
    say("sddmm", A.nnz, w)
    mat = _mat(A)
    d = torch.zeros(A.nnz, dtype=torch.float32, device=DEV)
    t = lambda a: torch.from_numpy(a).to(DEV)  # noqa: E731
    binding.frpca_sddmm(mat.h, w, t(P1), t(Q1), t(P2), t(Q2), d)
    rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
    c = A.col
    ref = (P1[rows].astype(np.float64) * Q1[c]).sum(1) + (P2[rows].astype(np.float64) * Q2[c]).sum(1)
    bound = (np.abs(P1[rows]) * np.abs(Q1[c])).sum(1) + (np.abs(P2[rows]) * np.abs(Q2[c])).sum(1)
    assert np.all(np.abs(np64(d) - ref) <= 1e-6 * bound + 1e-30)


def test_gather_probe_runs_and_checks_arguments():
    """The measurement helper behind the bench's row-gather ceiling: it reads whole waves of
    random rows (the count it reports), leaves a zero panel's sum unobserved and rejects panels
    narrower than a 512-byte row."""
    say("gather probe")
    mat = _mat(random_sparse(8, 8, 0.5, seed=1))
    P = torch.zeros((1000, 128), dtype=torch.float32, device=DEV)
    out = torch.full((64,), 3.0, dtype=torch.float32, device=DEV)
    ms, nr = binding.frpca_gather_probe(mat.h, P, 1000, 128, 5000, 1, out)
    assert ms > 0 and nr >= 5000 and nr % 2048 == 0
    assert torch.all(out == 3.0)
    with pytest.raises(binding.FrpcaError):
        binding.frpca_gather_probe(mat.h, P, 1000, 64, 5000, 1, out)
    mat.close()
