"""FP64 adjoint of the truncated SVD, projected onto the sparsity pattern of A.

The paper does not differentiate its method; the adjoint used here is the standard
reverse-mode rule of the SVD A = U S V^T (U m x k, V n x k, S diagonal, F_ij = 1/(s_j^2 -
s_i^2) for i != j, zero on the diagonal):

  Abar = U [ (F o (J - J^T)) S + diag(Sbar) + S (F o (K - K^T)) ] V^T
         + (Ubar - U J) S^+ V^T + U S^+ (Vbar - V K)^T,     J = U^T Ubar, K = V^T Vbar,

evaluated only at the stored nonzeros of A (a sparse A's values are the only free
parameters). It is exact when rank(A) = k with distinct singular values; for k < rank(A)
the Ubar and Vbar terms omit the coupling to the discarded triplets, while the Sbar term
(dsigma_i = u_i^T dA v_i) stays exact. Readings: F_ij = 0 where |s_j^2 - s_i^2| <=
gap_tol * s_1^2, and S^+ has 1/s_i or 0 where s_i = 0.

This is test infrastructure: only tests, the smoke check and the benchmark's CPU baseline
may use it.
"""
from __future__ import annotations

import numpy as np


def svd_adjoint_values(U, S, V, dU, dS, dV, rows, cols, gap_tol: float = 1e-12,
                       chunk: int = 1 << 20, center: bool = False) -> np.ndarray:
    """dL/dA at positions (rows[e], cols[e]) given dL/dU, dL/dS, dL/dV (None = zero).

    With center, U S V^T is the SVD of the column-centred matrix A - 1 mu^T (mu = column
    means of A, m = U.shape[0] rows): that map is A -> (I - 1 1^T / m) A, so dL/dA is the
    adjoint Abar of the centred matrix with each column's mean removed."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    k = S.size
    dU = np.zeros_like(U) if dU is None else np.asarray(dU, dtype=np.float64)
    dV = np.zeros_like(V) if dV is None else np.asarray(dV, dtype=np.float64)
    dS = np.zeros(k) if dS is None else np.asarray(dS, dtype=np.float64)
    J = U.T @ dU
    K = V.T @ dV
    s2 = S * S
    D = s2[None, :] - s2[:, None]
    ok = np.abs(D) > gap_tol * (s2.max() if k else 0.0)
    np.fill_diagonal(ok, False)
    F = np.zeros((k, k))
    np.divide(1.0, D, out=F, where=ok)
    sp = np.zeros(k)
    np.divide(1.0, S, out=sp, where=S > 0)
    M = (F * (J - J.T)) * S[None, :] + np.diag(dS) + S[:, None] * (F * (K - K.T))
    UM = U @ M
    Ur = (dU - U @ J) * sp[None, :]
    Vr = (dV - V @ K)
    Us = U * sp[None, :]
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    P = UM + Ur                                   # Abar = P V^T + Us Vr^T
    colmean = np.zeros(V.shape[0])
    if center:
        colmean = V @ P.mean(axis=0) + Vr @ Us.mean(axis=0)
    out = np.empty(rows.size)
    for a in range(0, rows.size, chunk):
        r = rows[a:a + chunk]
        c = cols[a:a + chunk]
        out[a:a + chunk] = (P[r] * V[c]).sum(1) + (Us[r] * Vr[c]).sum(1) - colmean[c]
    return out
