"""Helpers shared by the GPU parity tests (comparison metrics and device transfer)."""
from __future__ import annotations

import sys

import numpy as np

SIG_TOL = 1e-4    # relative singular-value error (FP32 path vs FP64 oracle)
ANG_TOL = 1e-3    # largest principal angle, radians (sine used; equal to 1e-9 relative here)
GAP_MIN = 1e-2    # relative Ritz gap below which a leading block is not separable


# pytest's capture manager, set by conftest: say() prints past the capture, so the steps of a
# long test (a full-size oracle run takes minutes) show as they happen
CAPTURE_MANAGER = None


def say(*a):
    capman = CAPTURE_MANAGER
    if capman is not None:
        with capman.global_and_fixture_disabled():
            print("[gpu-test]", *a, flush=True)
    else:
        print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def np64(t) -> np.ndarray:
    return t.detach().double().cpu().numpy()


def fp32_ulp_diff(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    ai = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    bi = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    return np.abs(ai - bi)


def sin_theta(Uref: np.ndarray, U: np.ndarray) -> float:
    if U.shape[1] == 0:
        return 0.0
    Q, _ = np.linalg.qr(U)
    Qr, _ = np.linalg.qr(Uref)
    return float(np.linalg.norm(Q - Qr @ (Qr.T @ Q), 2))


def separable_prefix(S_ritz: np.ndarray, k: int, gap_min: float = GAP_MIN) -> int:
    """Largest j <= k whose relative Ritz gap (s_j - s_{j+1}) / s_j is >= gap_min.

    S_ritz holds at least k+1 Ritz values (descending). The subspace of the leading j
    singular vectors is well conditioned only across such a gap (Davis-Kahan), so
    principal angles are compared on that prefix.
    """
    for j in range(k, 0, -1):
        if S_ritz[j - 1] > 0 and (S_ritz[j - 1] - S_ritz[j]) / S_ritz[j - 1] >= gap_min:
            return j
    return 0


def compare_triplets(Uo, So, Vo, Ug, Sg, Vg, S_ritz=None, sig_tol=SIG_TOL, ang_tol=ANG_TOL, gap_min=GAP_MIN):
    """Relative sigma error on all k and principal angles on the separable prefix."""
    k = So.size
    keep = So > 1e-6 * So.max() if So.max() > 0 else np.zeros(k, bool)
    sig_err = float(np.max(np.abs(Sg[keep] - So[keep]) / So[keep])) if keep.any() else 0.0
    zero_ok = bool(np.all(Sg[~keep] <= 1e-5 * max(So.max(), 1e-30)))
    j = k if S_ritz is None else separable_prefix(S_ritz, k, gap_min)
    su = sin_theta(Uo[:, :j], Ug[:, :j])
    sv = sin_theta(Vo[:, :j], Vg[:, :j])
    res = {"sig_err": sig_err, "sin_u": su, "sin_v": sv, "prefix": j, "zero_ok": zero_ok}
    res["ok"] = sig_err <= sig_tol and su <= ang_tol and sv <= ang_tol and zero_ok
    return res
