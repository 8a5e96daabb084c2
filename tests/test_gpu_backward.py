"""GPU adjoint (dL/d values through the truncated-SVD adjoint + SDDMM) against the FP64
dense formula and finite differences of an exact-SVD loss."""
import numpy as np
import pytest

import oracle
from gpu_util import np64, say
from synth import zipf_normal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1810_06825_amd import FrPCA, FrpcaError, binding, frpca_autograd  # noqa: E402

DEV = "cuda:0"


def _rows(A):
    return np.repeat(np.arange(A.m), np.diff(A.row_ptr))


@pytest.mark.parametrize("k,t", [(25, 30), (24, 31), (100, 40)])
def test_backward_matches_fp64_formula_at_gpu_factors(k, t):
    # k = 24 runs the SDDMM with four nonzeros per 16-byte gather (rows ending inside a group
    # of four); k = 25 the two-column-per-lane form; k = 100 the paired SDDMM and the
    # cross-Gram with seven 16-column tiles
    # (a pair and a single tile after the group of four) and the 112-deep panel product
    A = zipf_normal(m=20_000, n=4_000, t=t)
    q, s = 4, 10
    say("backward formula", k, A.m, A.n, A.nnz)
    mat = FrPCA.from_csr(A, device=DEV)
    U, S, V = mat.run(k, q, s, 11)
    rng = np.random.default_rng(0)
    dU = torch.from_numpy(rng.standard_normal((A.m, k)).astype(np.float32)).to(DEV)
    dV = torch.from_numpy(rng.standard_normal((A.n, k)).astype(np.float32)).to(DEV)
    dS = torch.from_numpy(rng.standard_normal(k).astype(np.float32)).to(DEV)
    for args in ((None, dS, None), (dU, None, None), (None, None, dV), (dU, dS, dV)):
        # frpca_backward rebuilds the run's factors; frpca_adjoint takes them from the caller
        dval = mat.backward(*args)
        dval_x = mat.adjoint(U, S, V, *args)
        ref = oracle.svd_adjoint_values(np64(U), np64(S), np64(V),
                                        *(None if a is None else np64(a) for a in args), _rows(A), A.col)
        err = np.abs(np64(dval) - ref).max() / np.abs(ref).max()
        err_x = np.abs(np64(dval_x) - ref).max() / np.abs(ref).max()
        say("  terms", [a is not None for a in args], "rel err", err, "explicit factors", err_x)
        assert err < 1e-4 and err_x < 1e-4
        # the rebuilt factors are the ones the run returned: both entry points agree to rounding
        assert np.abs(np64(dval) - np64(dval_x)).max() <= 1e-6 * np.abs(ref).max()
    mat.close()


def test_backward_needs_a_run():
    """frpca_backward refers to the handle's last run: none yet, or values changed since,
    is a state error; after a run it succeeds; frpca_adjoint works without a run."""
    A = zipf_normal(m=5_000, n=1_000, t=20)
    mat = FrPCA.from_csr(A, device=DEV)
    k = 10
    dS = torch.ones(k, device=DEV)
    with pytest.raises(FrpcaError) as ei:
        binding.frpca_backward(mat.h, None, dS, None, torch.empty(A.nnz, device=DEV))
    assert ei.value.code == binding.FRPCA_ESTATE
    U, S, V = mat.run(k, 3, 5, 1)
    g = mat.backward(None, dS, None)
    mat.set_values(mat.val.clone())
    with pytest.raises(FrpcaError) as ei:
        binding.frpca_backward(mat.h, None, dS, None, torch.empty(A.nnz, device=DEV))
    assert ei.value.code == binding.FRPCA_ESTATE
    # the explicit-factor adjoint is a pure function of its arguments
    g2 = mat.adjoint(U, S, V, None, dS, None)
    assert torch.allclose(g, g2, rtol=0, atol=1e-6 * float(g.abs().max()))
    # a later run with another k: backward follows the new run
    U3, S3, V3 = mat.run(12, 4, 4, 2)
    g3 = mat.backward(None, torch.ones(12, device=DEV), None)
    ref3 = oracle.svd_adjoint_values(np64(U3), np64(S3), np64(V3), None, np.ones(12), None, _rows(A), A.col)
    assert np.abs(np64(g3) - ref3).max() <= 1e-4 * np.abs(ref3).max()
    mat.close()


@pytest.mark.parametrize("k", [50, 51])
def test_backward_unaligned_k(k):
    """k not a multiple of 4 (the differentiated workload's k = 50): the panels are padded to
    16-byte rows; the result matches the FP64 formula with every term present."""
    A = zipf_normal(m=30_000, n=6_000, t=30)
    mat = FrPCA.from_csr(A, device=DEV)
    U, S, V = mat.run(k, 4, 10, 5)
    rng = np.random.default_rng(9)
    dU = torch.from_numpy(rng.standard_normal((A.m, k)).astype(np.float32)).to(DEV)
    dV = torch.from_numpy(rng.standard_normal((A.n, k)).astype(np.float32)).to(DEV)
    dS = torch.from_numpy(rng.standard_normal(k).astype(np.float32)).to(DEV)
    for args in ((dU, dS, None), (dU, dS, dV)):
        ref = oracle.svd_adjoint_values(np64(U), np64(S), np64(V),
                                        *(None if a is None else np64(a) for a in args), _rows(A), A.col)
        for dval in (mat.backward(*args), mat.adjoint(U, S, V, *args)):
            err = np.abs(np64(dval) - ref).max() / np.abs(ref).max()
            say("  k", k, "terms", [a is not None for a in args], "rel err", err)
            assert err < 1e-4
    mat.close()


def _exact_rank_sparse(m, n, k, seed):
    rng = np.random.default_rng(seed)
    Uf = rng.standard_normal((m, k)) * (rng.random((m, k)) < 0.3)
    Vf = rng.standard_normal((n, k)) * (rng.random((n, k)) < 0.3)
    D = (Uf * np.linspace(3, 1, k)) @ Vf.T
    D = D.astype(np.float32).astype(np.float64)
    from synth import from_dense

    return D, from_dense(D)


def test_backward_end_to_end_finite_differences():
    # rank-k input: the randomized forward is exact, the adjoint is exact, and the loss
    # sum(s) + sum_i w_i (c_i^T u_i)^2 is sign invariant, so FD of the exact-SVD loss applies
    m, n, k = 300, 200, 6
    D, A = _exact_rank_sparse(m, n, k, 3)
    rng = np.random.default_rng(4)
    C = rng.standard_normal((m, k))
    w = rng.random(k) + 0.5

    def loss_np(D_):
        U_, S_, Vt_ = np.linalg.svd(D_, full_matrices=False)
        U_ = U_[:, :k]
        return S_[:k].sum() + (w * ((C * U_).sum(0)) ** 2).sum()

    say("backward FD", A.nnz)
    mat = FrPCA.from_csr(A, device=DEV)
    vals = torch.from_numpy(A.val).to(DEV).requires_grad_(True)
    U, S, V = frpca_autograd(vals, mat, k, 4, 4, 21)
    Ct = torch.from_numpy(C.astype(np.float32)).to(DEV)
    wt = torch.from_numpy(w.astype(np.float32)).to(DEV)
    loss = S.sum() + (wt * ((Ct * U).sum(0)) ** 2).sum()
    loss.backward()
    g = np64(vals.grad)
    rows = _rows(A)
    idx = np.random.default_rng(5).choice(A.nnz, 80, replace=False)
    fd = []
    for e in idx:
        h = 1e-5 * max(abs(D[rows[e], A.col[e]]), 0.1)
        Dp, Dm = D.copy(), D.copy()
        Dp[rows[e], A.col[e]] += h
        Dm[rows[e], A.col[e]] -= h
        fd.append((loss_np(Dp) - loss_np(Dm)) / (2 * h))
    fd = np.array(fd)
    err = np.abs(g[idx] - fd).max() / np.abs(fd).max()
    say("  FD rel err", err)
    assert err < 1e-3
    mat.close()


def test_differentiated_workload_loss_is_sigma_sum_gradient():
    # loss = sum(sigma) + ||U_k W||^2: the second term is invariant, so dL/dvals equals
    # the closed form sum_i u_i[r] v_i[c]
    A = zipf_normal(m=50_000, n=10_000, t=30)
    k, q, s = 50, 4, 10
    say("differentiated loss", A.nnz)
    mat = FrPCA.from_csr(A, device=DEV)
    vals = torch.from_numpy(A.val).to(DEV).requires_grad_(True)
    U, S, V = frpca_autograd(vals, mat, k, q, s, 7)
    W = torch.from_numpy(np.random.default_rng(7).standard_normal((k, 8)).astype(np.float32)).to(DEV)
    loss = S.sum() + ((U @ W) ** 2).sum()
    loss.backward()
    Ug, Vg = np64(U), np64(V)
    ref = (Ug[_rows(A)] * Vg[A.col]).sum(1)
    err = np.abs(np64(vals.grad) - ref).max() / np.abs(ref).max()
    say("  rel err", err)
    assert err < 1e-4
    mat.close()
