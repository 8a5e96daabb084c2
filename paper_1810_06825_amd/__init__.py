"""Fast randomized PCA for sparse data (frPCA / frPCAt) on MI355X (gfx950).

Python face of the HIP library: ``FrPCA`` holds a CSR matrix resident on the GPU (with its
column-major mirror built once) and runs the randomized truncated SVD and its adjoint;
``frpca_autograd`` is a torch.autograd.Function returning dL/d(values). PyTorch only
provides device memory and the stream; every step runs in the library's kernels.
"""
from __future__ import annotations

import torch

from . import binding
from .binding import FrpcaError, FrpcaOpts, TIMER_NAMES  # noqa: F401

__all__ = ["FrPCA", "frpca_autograd", "FrpcaError", "binding"]


def _stream():
    return ctypes_void(torch.cuda.current_stream().cuda_stream)


def ctypes_void(x):
    import ctypes

    return ctypes.c_void_p(x)


class FrPCA:
    """A CSR matrix on the GPU prepared for frPCA (Alg. 5 / Alg. 6).

    row_ptr (int64[m+1]), col (int32[nnz]) and val (float32[nnz]) are CUDA tensors; they are
    kept referenced by the object because the library borrows them.
    """

    def __init__(self, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, shape,
                 panel_bf16: int = 0, sign_fix: bool = True, rank_tol: float = 0.0,
                 timing: bool = False, max_workspace: int = 0, center: bool = False,
                 gram_f32: bool = False, fused_pass: bool = False, final_f64: bool = False):
        assert row_ptr.is_cuda and col.is_cuda and val.is_cuda
        assert row_ptr.dtype == torch.int64 and col.dtype == torch.int32 and val.dtype == torch.float32
        self.row_ptr = row_ptr.contiguous()
        self.col = col.contiguous()
        self.val = val.contiguous()
        self.m, self.n = int(shape[0]), int(shape[1])
        self.nnz = int(self.col.numel())
        self.device = self.val.device
        opts = FrpcaOpts(int(panel_bf16), int(not sign_fix), float(rank_tol), int(timing), int(max_workspace),
                         int(center), int(gram_f32), int(fused_pass), int(final_f64))
        self.h = binding.frpca_create(self.m, self.n, self.nnz, self.row_ptr, self.col, self.val, opts,
                                      _stream())
        self.run_id = 0      # runs so far; frpca_backward refers to the last one
        self.last_k = 0

    @classmethod
    def from_csr(cls, A, device="cuda", **kw):
        """From an object with m, n, row_ptr, col, val numpy arrays (e.g. synth.Csr)."""
        rp = torch.from_numpy(A.row_ptr).to(device)
        col = torch.from_numpy(A.col).to(device)
        val = torch.from_numpy(A.val).to(device)
        return cls(rp, col, val, (A.m, A.n), **kw)

    def _sync_stream(self):
        binding.frpca_set_stream(self.h, _stream())

    def set_values(self, val: torch.Tensor):
        assert val.dtype == torch.float32 and val.numel() == self.nnz and val.device == self.device
        self.val = val.contiguous()
        self._sync_stream()
        binding.frpca_set_values(self.h, self.val)
        self.run_id += 1     # the last run's factors no longer describe the values

    def _panel(self, t, rows, cols, name, dtype=torch.float32):
        """Check a caller tensor against the shape, dtype and device the C ABI will assume."""
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if tuple(t.shape) != ((rows, cols) if cols is not None else (rows,)):
            want = (rows, cols) if cols is not None else (rows,)
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {want}")
        if t.dtype != dtype or t.device != self.device:
            raise ValueError(f"{name} must be {dtype} on {self.device}, got {t.dtype} on {t.device}")

    def run(self, k: int, passes: int, s: int, seed: int, out=None):
        """Rank-k truncated SVD (U m x k, S k descending, V n x k) with q = passes."""
        self._sync_stream()
        if out is None:
            U = torch.empty((self.m, k), dtype=torch.float32, device=self.device)
            S = torch.empty((k,), dtype=torch.float32, device=self.device)
            V = torch.empty((self.n, k), dtype=torch.float32, device=self.device)
        else:
            U, S, V = out
            for t, rows, cols, name in ((U, self.m, k, "U"), (S, k, None, "S"), (V, self.n, k, "V")):
                self._panel(t, rows, cols, name)
                if not t.is_contiguous():
                    raise ValueError(f"{name} must be contiguous (the library writes it in place)")
        binding.frpca_run(self.h, k, passes, s, seed, U, S, V)
        self.run_id += 1
        self.last_k = k
        return U, S, V

    def run_basic(self, k: int, power: int, s: int, seed: int, alg: int, out=None):
        """Rank-k truncated SVD by the basic randomized algorithm (Alg. 1 with alg = 1, Alg. 4
        with alg = 4) with `power` power steps and QR orthonormalisation (frpca_run_basic)."""
        self._sync_stream()
        if out is None:
            U = torch.empty((self.m, k), dtype=torch.float32, device=self.device)
            S = torch.empty((k,), dtype=torch.float32, device=self.device)
            V = torch.empty((self.n, k), dtype=torch.float32, device=self.device)
        else:
            U, S, V = out
            for t, rows, cols, name in ((U, self.m, k, "U"), (S, k, None, "S"), (V, self.n, k, "V")):
                self._panel(t, rows, cols, name)
                if not t.is_contiguous():
                    raise ValueError(f"{name} must be contiguous (the library writes it in place)")
        binding.frpca_run_basic(self.h, k, power, s, seed, alg, U, S, V)
        self.run_id += 1
        return U, S, V

    def eigsvds(self, k: int, s: int, seed: int, tol: float = 0.0, max_iter: int = 100):
        """Rank-k truncated SVD by eigSVDs (Alg. 3): the k largest eigenpairs of A^T A by a
        Chebyshev-filtered block subspace iteration (frpca_eigsvds). Returns (U, S, V, iters)."""
        self._sync_stream()
        U = torch.empty((self.m, k), dtype=torch.float32, device=self.device)
        S = torch.empty((k,), dtype=torch.float32, device=self.device)
        V = torch.empty((self.n, k), dtype=torch.float32, device=self.device)
        it = binding.frpca_eigsvds(self.h, k, s, seed, tol, max_iter, U, S, V)
        self.run_id += 1
        return U, S, V, it

    def _grads(self, k, dU, dS, dV):
        out = []
        for t, rows, cols, name in ((dU, self.m, k, "dU"), (dS, k, None, "dS"), (dV, self.n, k, "dV")):
            if t is not None:
                t = t.to(torch.float32)
                self._panel(t, rows, cols, name)
                t = t.contiguous()
            out.append(t)
        return out

    def backward(self, dU=None, dS=None, dV=None):
        """dL/d(values) (float32[nnz], CSR order) through the truncated-SVD adjoint at the
        factors of this object's last run (frpca_backward; None gradients are zero)."""
        self._sync_stream()
        dU, dS, dV = self._grads(self.last_k, dU, dS, dV)
        dval = torch.empty((self.nnz,), dtype=torch.float32, device=self.device)
        binding.frpca_backward(self.h, dU, dS, dV, dval)
        return dval

    def adjoint(self, U, S, V, dU=None, dS=None, dV=None):
        """The same adjoint at caller-given factors (frpca_adjoint)."""
        self._sync_stream()
        k = S.numel()
        U, S, V = (t.to(torch.float32) for t in (U, S, V))
        for t, rows, cols, name in ((U, self.m, k, "U"), (S, k, None, "S"), (V, self.n, k, "V")):
            self._panel(t, rows, cols, name)
        dU, dS, dV = self._grads(k, dU, dS, dV)
        dval = torch.empty((self.nnz,), dtype=torch.float32, device=self.device)
        binding.frpca_adjoint(self.h, k, U.contiguous(), S.contiguous(), V.contiguous(), dU, dS, dV, dval)
        return dval

    def info(self) -> dict:
        inf = binding.frpca_get_info(self.h)
        return {
            "m": inf.m, "n": inf.n, "nnz": inf.nnz, "orientation": inf.orientation, "k": inf.k,
            "s": inf.s, "passes": inf.passes, "rank_dropped": inf.rank_dropped,
            "workspace_bytes": inf.workspace_bytes, "create_ms": inf.create_ms,
            "hot_cols": inf.hot_cols, "row_blocks": inf.row_blocks, "hot_nnz": inf.hot_nnz,
            "t_ms": {n: inf.t_ms[i] for i, n in enumerate(TIMER_NAMES)},
            "t_count": {n: inf.t_count[i] for i, n in enumerate(TIMER_NAMES)},
        }

    def reset_timers(self):
        binding.frpca_reset_timers(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            binding.frpca_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _FrPCAFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, mat: FrPCA, k: int, passes: int, s: int, seed: int):
        # gradients of unused outputs stay None, so the adjoint skips their terms
        ctx.set_materialize_grads(False)
        mat.set_values(values.detach())
        U, S, V = mat.run(k, passes, s, seed)
        ctx.mat = mat
        ctx.run_id = mat.run_id
        ctx.save_for_backward(U, S, V)
        return U, S, V

    @staticmethod
    def backward(ctx, dU, dS, dV):
        U, S, V = ctx.saved_tensors
        mat = ctx.mat
        if mat.run_id == ctx.run_id:
            # the handle still holds this forward's factors
            dval = mat.backward(dU, dS, dV)
        else:
            # the handle ran again since: the adjoint at this forward's saved outputs
            dval = mat.adjoint(U, S, V, dU, dS, dV)
        return dval, None, None, None, None, None


def frpca_autograd(values: torch.Tensor, mat: FrPCA, k: int, passes: int, s: int, seed: int):
    """(U, S, V) = frPCA of the matrix with this pattern and these values; differentiable
    with respect to ``values`` through the library's adjoint + SDDMM kernels."""
    return _FrPCAFunction.apply(values, mat, k, passes, s, seed)
