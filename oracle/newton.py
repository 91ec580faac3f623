"""Inexact Newton-CG for the MAP point (Algorithm 1, Sec. 4.1).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Readings where the paper is silent or degenerate:
* norms are Euclidean 2-norms of nodal vectors; the outer loop stops when
  |g_i| <= rel_tol * |g_0| (or |g_i| <= abs_tol);
* eta_i = min(0.5, sqrt(|g_i| / |g_0|)) -- the printed eta_0 = 1 would accept
  mhat = 0 -- and CG always takes at least one iteration;
* CG is preconditioned with R^{-1} (the inverse regularization operator, Sec. 4.1),
  starts from mhat = 0 and stops when |H mhat + g| <= eta_i |g| (Eisenstat-Walker)
  or at non-positive curvature (Steihaug): at the first iteration the
  preconditioned steepest-descent direction is taken, later the current iterate;
* Armijo constant c = 1e-4 (the paper's interval is [1e-5, 1e-4]), step halving,
  at most 10 backtracks, at most 50 Newton and 500 CG iterations;
* the first gn_iters = 5 steps use the Gauss-Newton Hessian (positive
  semidefinite misfit part, the alternative the paper names where the full
  Hessian is not positive definite), later steps the full Hessian, which keeps
  the local superlinear convergence.
"""
from __future__ import annotations

import numpy as np

from .model import HESS_FULL, HESS_GN_FULL


def newton_cg(prob, m0=None, rel_tol=1e-6, abs_tol=0.0, max_iter=50, max_backtrack=10,
              c_armijo=1e-4, max_cg=500, gn_iters=5, verbose=False):
    """Returns (m, info) with info = dict(iters, cost, gnorm, cg_iters, alphas, converged, reason)."""
    m = prob.m_pr.copy() if m0 is None else np.array(m0, dtype=float)
    u = prob.forward(m)
    J, _, _ = prob.cost(m, u)
    info = dict(cost=[J], gnorm=[], cg_iters=[], alphas=[], converged=False, reason="max_iter")
    g0norm = None
    i = 0
    while i < max_iter:
        p = prob.adjoint(m, u)
        g = prob.gradient(m, u, p)
        gnorm = float(np.linalg.norm(g))
        info["gnorm"].append(gnorm)
        if g0norm is None:
            g0norm = gnorm
        if gnorm <= max(rel_tol * g0norm, abs_tol):
            info["converged"] = True
            info["reason"] = "gradient"
            break
        eta = min(0.5, np.sqrt(gnorm / g0norm))
        mode = HESS_GN_FULL if i < gn_iters else HESS_FULL

        # --- CG with Steihaug and Eisenstat-Walker termination ---
        def H(v):
            return prob.hessian_apply(m, u, p, v, mode)

        mhat = np.zeros_like(m)
        r = -g.copy()
        z = prob.R_solve(r)
        d = z.copy()
        rz = float(r @ z)
        ncg = 0
        for k in range(max_cg):
            Hd = H(d)
            dHd = float(d @ Hd)
            ncg += 1
            if dHd <= 0.0:
                if k == 0:
                    mhat = d.copy()
                break
            alpha = rz / dHd
            mhat = mhat + alpha * d
            r = r - alpha * Hd
            if np.linalg.norm(r) <= eta * gnorm:
                break
            z = prob.R_solve(r)
            rz_new = float(r @ z)
            d = z + (rz_new / rz) * d
            rz = rz_new
        info["cg_iters"].append(ncg)

        # --- Armijo backtracking ---
        gm = float(g @ mhat)
        alpha = 1.0
        accepted = False
        for _ in range(max_backtrack):
            m_try = m + alpha * mhat
            u_try = prob.forward(m_try)
            J_try, _, _ = prob.cost(m_try, u_try)
            if J_try < J + alpha * c_armijo * gm:
                m, u, J = m_try, u_try, J_try
                accepted = True
                break
            alpha *= 0.5
        info["alphas"].append(alpha)
        info["cost"].append(J)
        if verbose:
            print(f"newton {i}: J={J:.6e} |g|={gnorm:.3e} cg={ncg} alpha={alpha}")
        if not accepted:
            info["reason"] = "line_search"
            break
        i += 1
    info["iters"] = i
    return m, info
