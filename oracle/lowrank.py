"""Randomized generalized eigensolver and low-rank posterior sampling.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* PreCholQR (Algorithm 4): Householder QR of Y, B-Gram of the orthonormal
  factor, Cholesky, triangular solve.
* Double-pass randomized eigensolver (Algorithm 2) for A v = lambda B v with
  A = H_misfit and B = R (Sec. 4.2, Eq. eq:eigenproblem_1).
* Single-pass randomized eigensolver (Algorithm 3): T from the first pass
  alone, as the least-squares solution over symmetric matrices of
  T (Qbar^T Omega) = Qbar^T Y (Eq. eq:Tsinglepass), Qbar = B Q.
* The single-pass T of Saibaba, Lee & Kitanidis that Sec. 4.2 compares with
  (a baseline for the comparison of Fig. 2 only).
* Posterior sample y = (I - V_r S_r V_r^T R) x with S_r = I - (Lambda_r + I)^{-1/2}
  (Sec. 4.3.2, Eq. eq:sample_post).
* Pointwise variance (Sec. 4.4): the prior's diag(R^-1) from a randomized
  eigendecomposition of R^-1 (Eq. eq:prior_mvar), the posterior's by the
  low-rank correction (Eq. eq:post_mvar), and the stochastic estimator of
  Bekas, Kokiopoulou & Saad the section compares with (Eq.
  eq:stoc_diag_estimator).

Readings: T is symmetrized as (T + T^T)/2 before its eigendecomposition and the
eigenpairs are sorted by decreasing eigenvalue.  In Algorithm 3 the norm of the
least-squares problem is the Frobenius norm and the constraint set is the
symmetric matrices (the semidefinite restriction is not imposed: for the
Gauss-Newton misfit Hessian T is semidefinite up to rounding, and only its
leading eigenpairs are kept).  The Saibaba-Lee-Kitanidis formula is printed
as (Q^T B Omega)^-1 (Q^T B Y) (Q^T B Omega)^-1, which does not approximate
Q^T A Q; it is read as W^-T (Omega^T Ybar) W^-1 with W = Q^T B Omega and
Ybar = A Omega, the symmetric form that follows from A ~ B Q T Q^T B.
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


def _eig_desc(T, k):
    lam, S = np.linalg.eigh(0.5 * (T + T.T))
    order = np.argsort(lam)[::-1]
    return lam[order], S[:, order]


def symmetric_least_squares(W, Z):
    """argmin over symmetric X of |X W - Z|_F (W, Z: s x s), written as an ordinary
    least-squares problem in the s (s + 1) / 2 entries of the upper triangle:
    X = sum_{i <= j} x_ij E_ij with E_ij = e_i e_j^T + e_j e_i^T (i < j) or
    e_i e_i^T, so X W = sum x_ij E_ij W and the columns of the system are
    vec(E_ij W)."""
    s = W.shape[0]
    cols, pairs = [], []
    for i in range(s):
        for j in range(i, s):
            E = np.zeros((s, s))
            E[i, j] = 1.0
            E[j, i] = 1.0
            cols.append((E @ W).reshape(-1))
            pairs.append((i, j))
    A = np.column_stack(cols)
    x, *_ = np.linalg.lstsq(A, Z.reshape(-1), rcond=None)
    X = np.zeros((s, s))
    for (i, j), v in zip(pairs, x):
        X[i, j] = v
        X[j, i] = v
    return X


def single_pass(A_apply, B_apply, Binv_apply, Omega, k):
    """Algorithm 3.  Omega: (n, k+p) Gaussian.  Returns (lmbda[k], V[n, k], extras).

    One pass of A over Omega: Ybar = A Omega, Y = B^-1 Ybar; PreCholQR gives Q
    (Q^T B Q = I) and Qbar = B Q (Qbar^T B^-1 Qbar = I); T is the symmetric
    least-squares solution of T (Qbar^T Omega) = Qbar^T Y; V = Q S_k.
    """
    s = Omega.shape[1]
    Ybar = np.column_stack([A_apply(Omega[:, j]) for j in range(s)])
    Y = np.column_stack([Binv_apply(Ybar[:, j]) for j in range(s)])
    Q, Qbar, _ = pre_chol_qr(Y, B_apply)
    W = Qbar.T @ Omega
    Z = Qbar.T @ Y
    T = symmetric_least_squares(W, Z)
    lam, S = _eig_desc(T, k)
    return lam[:k], Q @ S[:, :k], dict(Q=Q, Qbar=Qbar, T=T, W=W, Z=Z, lam_all=lam, Ybar=Ybar)


def single_pass_slk(A_apply, B_apply, Binv_apply, Omega, k):
    """Single-pass T of Saibaba, Lee & Kitanidis as compared in Sec. 4.2 (reading
    in the module docstring): T = W^-T (Omega^T Ybar) W^-1, W = Q^T B Omega."""
    s = Omega.shape[1]
    Ybar = np.column_stack([A_apply(Omega[:, j]) for j in range(s)])
    Y = np.column_stack([Binv_apply(Ybar[:, j]) for j in range(s)])
    Q, Qbar, _ = pre_chol_qr(Y, B_apply)
    W = Qbar.T @ Omega
    M = Omega.T @ Ybar
    T = np.linalg.solve(W.T, np.linalg.solve(W.T, M).T).T   # W^-T M W^-1 (M symmetric)
    lam, S = _eig_desc(T, k)
    return lam[:k], Q @ S[:, :k], dict(Q=Q, T=T, lam_all=lam)


def prior_variance(Rinv_apply, Omega):
    """Eq. eq:prior_mvar: diag(R^-1) ~ sum_i mu_i vbar_i (.) vbar_i with (mu_i, vbar_i)
    the eigenpairs of R^-1 from Algorithm 2 with A = R^-1, B = I and no
    oversampling (Omega: n x rbar).  Returns (diag, mu)."""
    ident = lambda v: np.array(v, dtype=float)
    mu, Vb, _ = double_pass(Rinv_apply, ident, ident, Omega, Omega.shape[1])
    return (Vb * Vb) @ mu, mu


def posterior_variance(prior_diag, V, lam):
    """Eq. eq:post_mvar: diag(H^-1) ~ diag(R^-1) - sum_i lambda_i / (1 + lambda_i) v_i (.) v_i."""
    lam = np.asarray(lam, dtype=float)
    return prior_diag - (V * V) @ (lam / (1.0 + lam))


def stochastic_diagonal(Rinv_apply, Z):
    """Eq. eq:stoc_diag_estimator (Bekas, Kokiopoulou & Saad): diag(R^-1) ~
    [sum_j z_j (.) w_j] (/) [sum_j z_j (.) z_j] with R w_j = z_j; Z: n x s."""
    W = np.column_stack([Rinv_apply(Z[:, j]) for j in range(Z.shape[1])])
    return (Z * W).sum(axis=1) / (Z * Z).sum(axis=1)


def posterior_sample_update(x, V, lam, R_apply):
    """y = (I - V S V^T R) x, S = diag(1 - 1/sqrt(1 + lambda)) (Eq. eq:sample_post).  Needs lambda > -1."""
    lam = np.asarray(lam, dtype=float)
    if np.any(lam <= -1.0):
        raise ValueError("posterior sampling needs every eigenvalue > -1")
    s = 1.0 - 1.0 / np.sqrt(1.0 + lam)
    Rx = R_apply(x)
    return x - V @ (s * (V.T @ Rx))
