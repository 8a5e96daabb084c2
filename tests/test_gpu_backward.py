"""GPU adjoint (dL/d values through the truncated-SVD adjoint + SDDMM) against the FP64
dense formula and finite differences of an exact-SVD loss."""
import numpy as np
import pytest

import oracle
from gpu_util import np64, say
from synth import zipf_normal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1810_06825_amd import FrPCA, frpca_autograd  # noqa: E402

DEV = "cuda:0"


def _rows(A):
    return np.repeat(np.arange(A.m), np.diff(A.row_ptr))


@pytest.mark.parametrize("k,t", [(25, 30), (24, 31), (100, 40)])
def test_backward_matches_fp64_formula_at_gpu_factors(k, t):
    # k = 24 runs the paired 16-byte SDDMM (odd row lengths leave a single last entry);
    # k = 25 the two-column-per-lane form; k = 100 the cross-Gram with seven 16-column tiles
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
        dval = mat.backward(U, S, V, *args)
        ref = oracle.svd_adjoint_values(np64(U), np64(S), np64(V),
                                        *(None if a is None else np64(a) for a in args), _rows(A), A.col)
        err = np.abs(np64(dval) - ref).max() / np.abs(ref).max()
        say("  terms", [a is not None for a in args], "rel err", err)
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
