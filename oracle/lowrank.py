"""Randomized generalized eigensolver and low-rank posterior sampling.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* PreCholQR (Algorithm 4): Householder QR of Y, B-Gram of the orthonormal
  factor, Cholesky, triangular solve.
* Double-pass randomized eigensolver (Algorithm 2) for A v = lambda B v with
  A = H_misfit and B = R (Sec. 4.2, Eq. eq:eigenproblem_1).
* Posterior sample y = (I - V_r S_r V_r^T R) x with S_r = I - (Lambda_r + I)^{-1/2}
  (Sec. 4.3.2, Eq. eq:sample_post).

Readings: T is symmetrized as (T + T^T)/2 before its eigendecomposition and the
eigenpairs are sorted by decreasing eigenvalue.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def pre_chol_qr(Y, B_apply):
    """Algorithm 4.  Y: (n, s).  Returns (Q, Qbar, Rfac) with Q^T B Q = I, Y = Q Rfac."""
    Z, RY = np.linalg.qr(Y, mode="reduced")            # Householder (LAPACK geqrf)
    Zbar = np.column_stack([B_apply(Z[:, j]) for j in range(Z.shape[1])])
    RZ = sla.cholesky(Z.T @ Zbar, lower=False)         # upper triangular, R_Z^T R_Z = Z^T B Z
    Q = sla.solve_triangular(RZ, Z.T, trans="T", lower=False).T   # Z R_Z^{-1}
    Qbar = sla.solve_triangular(RZ, Zbar.T, trans="T", lower=False).T
    return Q, Qbar, RZ @ RY


def double_pass(A_apply, B_apply, Binv_apply, Omega, k):
    """Algorithm 2.  Omega: (n, k+p) Gaussian.  Returns (lmbda[k], V[n, k], extras)."""
    s = Omega.shape[1]
    Ybar = np.column_stack([A_apply(Omega[:, j]) for j in range(s)])
    Y = np.column_stack([Binv_apply(Ybar[:, j]) for j in range(s)])
    Q, _, _ = pre_chol_qr(Y, B_apply)
    AQ = np.column_stack([A_apply(Q[:, j]) for j in range(s)])
    T = Q.T @ AQ
    T = 0.5 * (T + T.T)
    lam, S = np.linalg.eigh(T)
    order = np.argsort(lam)[::-1]
    lam, S = lam[order], S[:, order]
    V = Q @ S[:, :k]
    return lam[:k], V, dict(Q=Q, T=T, lam_all=lam, Y=Y)


def posterior_sample_update(x, V, lam, R_apply):
    """y = (I - V S V^T R) x, S = diag(1 - 1/sqrt(1 + lambda)) (Eq. eq:sample_post).  Needs lambda > -1."""
    lam = np.asarray(lam, dtype=float)
    if np.any(lam <= -1.0):
        raise ValueError("posterior sampling needs every eigenvalue > -1")
    s = 1.0 - 1.0 / np.sqrt(1.0 + lam)
    Rx = R_apply(x)
    return x - V @ (s * (V.T @ Rx))
