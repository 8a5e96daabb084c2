"""The allocation-free eigendecomposition (frpca_eig_noalloc) against frpca_eig, through the
C-ABI: two calls in a row on the shared static scratch, the second with a smaller matrix, each
bitwise equal to the allocating entry point and at FP64 accuracy against LAPACK; sizes past the
static buffer's limit are rejected. Runs alone in a fresh process or after the other tests.
"""
import numpy as np
import pytest

from gpu_util import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1810_06825_amd import FrPCA, FrpcaError, binding  # noqa: E402
from synth import random_sparse  # noqa: E402

DEV = "cuda:0"


def _sym(l, seed):
    rng = np.random.default_rng(seed)
    Q = np.linalg.qr(rng.standard_normal((l, l)))[0]
    d = np.geomspace(1e-6, 1e4, l) * rng.choice([-1.0, 1.0], l)
    G = (Q * d) @ Q.T
    return 0.5 * (G + G.T)


def _decompose(fn, l, G):
    Gd = torch.from_numpy(G).to(DEV)
    W = torch.full((l, l), np.nan, dtype=torch.float64, device=DEV)
    d = torch.full((l,), np.nan, dtype=torch.float64, device=DEV)
    fn(l, Gd, W, d)
    torch.cuda.synchronize()
    return W.cpu().numpy(), d.cpu().numpy()


def test_eig_noalloc_matches_eig_twice():
    mat = FrPCA.from_csr(random_sparse(8, 8, 0.5, seed=1), device=DEV)
    stream = torch.cuda.current_stream().cuda_stream
    for l, seed in ((120, 31), (37, 32)):   # the second call is smaller than the first
        say("eig_noalloc", l)
        G = _sym(l, seed)
        W0, d0 = _decompose(lambda l_, G_, W_, d_: binding.frpca_eig(mat.h, l_, G_, W_, d_), l, G)
        W1, d1 = _decompose(lambda l_, G_, W_, d_: binding.frpca_eig_noalloc(l_, G_, W_, d_, stream), l, G)
        assert np.array_equal(d1, d0) and np.array_equal(W1, W0)
        nrm = np.abs(d1).max()
        assert np.abs(d1 - np.linalg.eigvalsh(G)).max() <= 1e-12 * nrm
        assert np.abs(G @ W1 - W1 * d1).max() <= 1e-12 * nrm
        assert np.abs(W1.T @ W1 - np.eye(l)).max() <= 1e-12
    mat.close()


def test_eig_noalloc_rejects_sizes_past_its_buffer():
    G = torch.zeros((129, 129), dtype=torch.float64, device=DEV)
    W = torch.zeros_like(G)
    d = torch.zeros(129, dtype=torch.float64, device=DEV)
    for l in (129, 0):
        with pytest.raises(FrpcaError) as ei:
            binding.frpca_eig_noalloc(l, G, W, d)
        assert ei.value.code == binding.FRPCA_EINVAL
        assert "1..128" in str(ei.value)
