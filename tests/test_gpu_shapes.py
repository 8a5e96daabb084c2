"""frpca_run against the FP64 oracle over a seeded spread of shapes and options: tall, wide and
square matrices, l from 2 to 128, s = 0, every pass count from 2 to 7, structurally empty rows
and columns, integer values, the BF16 and centred modes. The GPU and the oracle draw the same
Gaussian matrices, so the comparison measures only the numerics (the oracle's own accuracy
against the exact SVD is pinned elsewhere).
"""
import numpy as np
import pytest
import scipy.sparse

import oracle
from gpu_util import ANG_TOL, SIG_TOL, compare_triplets, np64, say
from synth import random_sparse

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1810_06825_amd import FrPCA  # noqa: E402

DEV = "cuda:0"


def _cases():
    rng = np.random.default_rng(20181015)
    out = []
    shapes = [(3000, 800), (700, 2600), (1500, 1500), (130, 4000), (5000, 129), (2048, 512),
              (999, 1001), (4000, 300), (300, 300), (6000, 2000), (1200, 140), (160, 1700)]
    for i, (m, n) in enumerate(shapes):
        short = min(m, n)
        l = int(rng.integers(2, min(128, short) + 1))
        k = int(rng.integers(1, l + 1))
        if i == 2:
            l, k = 128, 100  # the widest sketch
        if i == 5:
            k = l            # no oversampling
        s = l - k
        q = 2 + i % 6
        density = min(0.2, 60_000 / (m * n) * 3)
        empty_rows = tuple(rng.choice(m, size=min(5, m // 50), replace=False)) if i % 3 == 0 else ()
        empty_cols = tuple(rng.choice(n, size=min(5, n // 50), replace=False)) if i % 4 == 1 else ()
        kw = {}
        if i % 5 == 2:
            kw["center"] = True
        if i % 7 == 3:
            kw["panel_bf16"] = 4
        out.append((i, m, n, k, s, q, density, empty_rows, empty_cols, i % 2 == 1, kw))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"{c[1]}x{c[2]}-k{c[3]}-s{c[4]}-q{c[5]}")
def test_shape_spread_matches_oracle(case):
    i, m, n, k, s, q, density, er, ec, integer, kw = case
    A = random_sparse(m, n, density, seed=100 + i, empty_rows=er, empty_cols=ec, integer_values=integer)
    say("shape spread", m, n, A.nnz, f"k={k} s={s} q={q}", kw)
    mat = FrPCA.from_csr(A, device=DEV, **kw)
    U, S, V = mat.run(k, q, s, 7 + i)
    torch.cuda.synchronize()
    Ug, Sg, Vg = np64(U), np64(S), np64(V)
    mat.close()
    center = bool(kw.get("center"))
    Uo, So, Vo, _ = oracle.frpca(A, k, q, s, 7 + i, center=center)
    S_ritz = oracle.frpca(A, k + 1, q, s - 1, 7 + i, center=center)[1] if s >= 1 else None
    # BF16 panels (mode 4: the long-side panel of all but the last pass pair) are bounded by the
    # BF16 rounding unit, the rest by the FP32 tolerances
    bf = "panel_bf16" in kw
    r = compare_triplets(Uo, So, Vo, Ug, Sg, Vg, S_ritz, 2.0 ** -9 if bf else SIG_TOL, 2.0 ** -6 if bf else ANG_TOL)
    say("  ->", {kk: (round(v, 9) if isinstance(v, float) else v) for kk, v in r.items()})
    assert r["ok"], r
    # by construction the long-side factor is the operator applied to the short-side one over S
    # (Alg. 6: U = A Q W / S with V = Q W, so A V = U S; Alg. 5: V = A^T Q W / S with U = Q W, so
    # A^T U = V S), a check on the GPU factors that needs no separable prefix; for the centred
    # mode the operator is A - 1 mu^T
    Ad = scipy.sparse.csr_matrix((A.val.astype(np.float64), A.col, A.row_ptr), shape=(m, n))
    mu = np.asarray(Ad.mean(axis=0)).ravel() if center else np.zeros(n)
    if m >= n:
        lhs, rhs = Ad @ Vg - np.outer(np.ones(m), mu @ Vg), Ug * Sg
    else:
        lhs, rhs = Ad.T @ Ug - np.outer(mu, Ug.sum(axis=0)), Vg * Sg
    res = np.abs(lhs - rhs).max() / max(Sg.max(), 1e-30)
    say(f"  max |op(short factor) - long factor S| / sigma_1 = {res:.2e}")
    assert res < 1e-6
    # orthonormal factors where the spectrum is nonzero, descending values
    assert np.all(np.diff(Sg) <= 0)
    nz = Sg > 1e-5 * max(Sg.max(), 1e-30)
    for M in (Ug[:, nz], Vg[:, nz]):
        assert np.abs(M.T @ M - np.eye(M.shape[1])).max() < 1e-4
