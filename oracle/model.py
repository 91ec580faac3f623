"""Poisson coefficient inversion: forward, adjoint, gradient and Hessian action.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Discrete counterparts of the paper's formulas, with sparse direct solves:

* forward problem  -div(e^m grad u) = 0, u = 0 on y = 0, u = 1 on y = 1,
  zero flux on x = 0 and x = 1 (Sec. 5.1, Eq. equ:poi and eq:poisson_weak);
* cost  J(m) = 1/2 sigma^-2 |B u - d|^2 + 1/2 (m - m_pr)^T R (m - m_pr)
  (Eq. eq:cost-elliptic, discretized as in Sec. 2.3);
* adjoint and gradient (Appendix A, Eqs. eq:firstadj and eq:firstcontrol);
* incremental forward/adjoint and the Hessian action (Appendix A,
  Eqs. eq:incrementals1, eq:incrementals2, eq:incrementals3; abstract form in
  Sec. 2.1, Eq. eq:abstract_hessianAction);
* bilaplacian prior C = A^{-2}, A = -gamma div(Theta grad) + delta I with a
  Robin condition (Sec. 5.1, Eq. eq:PoissonPrior; Sec. 2.2), discretized as
  R = K_A M^{-1} K_A with K_A = gamma K_Theta + delta M + beta M_boundary;
* prior sampling R x = C eta through the rectangular factor (Sec. 4.3.1,
  Eq. eq:sample_prior, and Appendix C).  With R = K_A M^{-1} K_A the factor is
  C = K_A M^{-1} C_M, so x = K_A^{-1} C_M eta.

Derivatives are those of the discrete cost (centroid quadrature of e^m): for a
triangle T with vertices (a, r, b),
    d c_T / d m_v = c_T / 3,   d^2 c_T / d m_v d m_w = c_T / 9   (v, w in T),
so the gradient and Hessian actions below are exact derivatives of J.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import mesh as msh
from . import p2 as p2sp

HESS_FULL = 0        # full Hessian of J (misfit + prior)
HESS_MISFIT = 1      # data-misfit part only
HESS_GN_FULL = 2     # Gauss-Newton misfit + prior
HESS_GN_MISFIT = 3   # Gauss-Newton misfit only


def default_beta(gamma: float, delta: float) -> float:
    """Robin coefficient beta = sqrt(gamma delta) / 1.42 (a reading: the paper gives only beta ~ sqrt(gamma delta))."""
    return np.sqrt(gamma * delta) / 1.42


class P1State:
    """Linear state space: the parameter's own nodes (the workloads' default)."""

    def __init__(self, mesh: msh.Mesh, geo: msh.Geometry):
        self.mesh, self.geo = mesh, geo
        self.n = mesh.n
        self.free = mesh.free
        self.uD = np.zeros(mesh.n)
        self.uD[mesh.xy[:, 1] == 1.0] = 1.0

    def stiffness(self, cT):
        return msh.stiffness(self.mesh, self.geo, cT)

    def tri_forms(self, v, w):
        """Per-triangle |T| grad(v) . grad(w) for nodal vectors v, w (unit coefficient)."""
        G = self.geo.grads                         # (nt, 3, 2)
        gv = np.einsum('tai,ta->ti', G, v[self.mesh.tris])
        gw = np.einsum('tai,ta->ti', G, w[self.mesh.tris])
        return self.geo.area * np.einsum('ti,ti->t', gv, gw)

    def observation_operator(self, pts):
        return msh.observation_operator(self.mesh, pts)


class Problem:
    """One instance of the discrete coefficient-inversion problem.

    state_degree 1: P1 state on the parameter's nodes; 2: P2 state (the
    paper's Sec. 5.1 pairing), vectors u, p, uhat, phat then live on the
    (2N+1)^2 nodes of ``p2.P2Space`` while m, g and H mhat stay P1."""

    def __init__(self, N: int, gamma: float, delta: float, m_prior: float = -2.0,
                 beta: float | None = None, Theta: np.ndarray | None = None,
                 obs_xy: np.ndarray | None = None, d_obs: np.ndarray | None = None,
                 sigma: float = 0.01, state_degree: int = 1):
        self.mesh = msh.Mesh(N)
        self.geo = msh.Geometry(self.mesh)
        self.N = N
        self.n = self.mesh.n
        if state_degree not in (1, 2):
            raise ValueError("state_degree must be 1 or 2")
        self.state_degree = state_degree
        self.S = P1State(self.mesh, self.geo) if state_degree == 1 else p2sp.P2Space(self.mesh, self.geo)
        self.ns = self.S.n
        self.gamma, self.delta = float(gamma), float(delta)
        self.beta = default_beta(gamma, delta) if beta is None else float(beta)
        self.Theta = None if Theta is None else np.asarray(Theta, dtype=float)
        self.m_pr = np.full(self.n, float(m_prior))
        self.sigma = float(sigma)
        # prior operators (parameter space: every node is a dof, Robin boundary)
        K = msh.stiffness(self.mesh, self.geo, np.ones(self.mesh.tris.shape[0]), self.Theta)
        self.M = msh.mass(self.mesh, self.geo).tocsc()
        self.Mb = msh.boundary_mass(self.mesh)
        self.KA = (self.gamma * K + self.delta * self.M + self.beta * self.Mb).tocsc()
        # factorizations of K_A and M and the mass factor C_M are built at first use
        self._KA_lu_, self._M_lu_, self._CM = None, None, None
        # state boundary data
        self.free = self.S.free
        self.uD = self.S.uD
        self.set_observations(obs_xy, d_obs)
        self._fact_m = None  # cache of (m, c_T, A, LU of A_FF)

    # -- observations ---------------------------------------------------------
    def set_observations(self, obs_xy, d_obs):
        if obs_xy is None:
            self.B = sp.csr_matrix((0, self.ns))
            self.d = np.zeros(0)
            return
        self.obs_xy = np.asarray(obs_xy, dtype=float)
        self.B = self.S.observation_operator(self.obs_xy)
        self.d = np.zeros(self.B.shape[0]) if d_obs is None else np.asarray(d_obs, dtype=float)

    # -- prior (Sec. 5.1, Sec. 2.3) -------------------------------------------
    @property
    def _KA_lu(self):
        if self._KA_lu_ is None:
            self._KA_lu_ = spla.splu(self.KA)
        return self._KA_lu_

    @property
    def _M_lu(self):
        if self._M_lu_ is None:
            self._M_lu_ = spla.splu(self.M)
        return self._M_lu_

    @property
    def CM(self):
        """Rectangular mass factor C_M (n x 6 N^2), C_M C_M^T = M (Appendix C)."""
        if self._CM is None:
            self._CM = msh.mass_factor(self.mesh, self.geo)
        return self._CM

    def M_solve(self, x):
        return self._M_lu.solve(np.asarray(x, dtype=float))

    def KA_solve(self, x):
        return self._KA_lu.solve(np.asarray(x, dtype=float))

    def R_apply(self, x):
        """R x = K_A M^{-1} K_A x."""
        return self.KA @ self.M_solve(self.KA @ x)

    def R_solve(self, x):
        """R^{-1} x = K_A^{-1} M K_A^{-1} x."""
        return self.KA_solve(self.M @ self.KA_solve(x))

    def prior_sample(self, eta):
        """m_pr + K_A^{-1} C_M eta: a draw from N(m_pr, R^{-1}) (Eq. eq:sample_prior)."""
        return self.m_pr + self.KA_solve(self.CM @ eta)

    # -- state operator A(m) ---------------------------------------------------
    def _factor(self, m):
        m = np.asarray(m, dtype=float)
        if self._fact_m is not None and np.array_equal(self._fact_m[0], m):
            return self._fact_m
        cT = msh.coefficient(self.mesh, m)
        A = self.S.stiffness(cT).tocsr()
        f = self.free
        AFF = A[f][:, f].tocsc()
        lu = spla.splu(AFF)
        self._fact_m = (m.copy(), cT, A, lu)
        return self._fact_m

    def stiffness(self, m):
        return self._factor(m)[2]

    def coefficient(self, m):
        return self._factor(m)[1]

    def _solve_free(self, m, rhs_free):
        return self._factor(m)[3].solve(rhs_free)

    # -- forward, cost (Alg. 1 inputs) ----------------------------------------
    def forward(self, m, f_load=None):
        """u with u_D on the Dirichlet nodes and A_FF u_F = b_F - A_FD u_D."""
        _, _, A, _ = self._factor(m)
        f = self.free
        rhs = -(A @ self.uD)
        if f_load is not None:
            rhs = rhs + f_load
        u = self.uD.copy()
        u[f] = self._solve_free(m, rhs[f])
        return u

    def misfit(self, u):
        r = self.B @ u - self.d
        return 0.5 * float(r @ r) / self.sigma ** 2

    def regularization(self, m):
        dm = m - self.m_pr
        return 0.5 * float(dm @ self.R_apply(dm))

    def cost(self, m, u=None):
        if u is None:
            u = self.forward(m)
        mis = self.misfit(u)
        reg = self.regularization(m)
        return mis + reg, mis, reg

    # -- adjoint and gradient (Appendix A) ------------------------------------
    def adjoint(self, m, u):
        """A_FF p_F = -[B^T (B u - d)]_F / sigma^2, p = 0 on the Dirichlet nodes (Eq. eq:firstadj)."""
        rhs = -(self.B.T @ (self.B @ u - self.d)) / self.sigma ** 2
        p = np.zeros(self.ns)
        # A(m) is symmetric, so the adjoint operator is A_FF itself
        p[self.free] = self._solve_free(m, rhs[self.free])
        return p

    def _tri_forms(self, v, w):
        """Per-triangle int_T grad(v) . grad(w) for state vectors v, w (unit coefficient)."""
        return self.S.tri_forms(v, w)

    def _vertex_sum(self, per_tri):
        """Scatter per-triangle values to their three vertices (sum)."""
        out = np.zeros(self.n)
        for a in range(3):
            np.add.at(out, self.mesh.tris[:, a], per_tri)
        return out

    def gradient(self, m, u, p):
        """g = R (m - m_pr) + C(u)^T p, with (C(u)^T p)_v = sum_{T∋v} (c_T/3) |T| grad u . grad p (Eq. eq:firstcontrol)."""
        cT = self.coefficient(m)
        g_data = self._vertex_sum(cT / 3.0 * self._tri_forms(u, p))
        return self.R_apply(m - self.m_pr) + g_data

    # -- incremental problems and Hessian action (Appendix A) -----------------
    def _sens_apply(self, cT, mhat, w):
        """C(w) mhat = sum_T s_T |T| grad(phi) . grad(w_T), s_T = (c_T/3) sum_{v in T} mhat_v.

        This is the derivative of A(m) w in direction mhat (a stiffness matrix with
        per-triangle coefficient s_T applied to w).
        """
        sT = cT / 3.0 * mhat[self.mesh.tris].sum(axis=1)
        Ks = self.S.stiffness(sT)
        return Ks @ w

    def inc_forward(self, m, u, mhat):
        """A_FF uhat_F = -[C(u) mhat]_F, uhat_D = 0 (Eq. eq:incrementals1)."""
        cT = self.coefficient(m)
        rhs = -self._sens_apply(cT, mhat, u)
        uh = np.zeros(self.ns)
        uh[self.free] = self._solve_free(m, rhs[self.free])
        return uh

    def inc_adjoint(self, m, p, mhat, uhat, gauss_newton=False):
        """A_FF phat_F = -[B^T B uhat / sigma^2 + C(p) mhat]_F, phat_D = 0 (Eq. eq:incrementals2).

        Gauss-Newton drops the C(p) mhat term (footnote to Eq. eq:laplace_approx).
        """
        cT = self.coefficient(m)
        rhs = -(self.B.T @ (self.B @ uhat)) / self.sigma ** 2
        if not gauss_newton:
            rhs = rhs - self._sens_apply(cT, mhat, p)
        ph = np.zeros(self.ns)
        ph[self.free] = self._solve_free(m, rhs[self.free])
        return ph

    def hessian_apply(self, m, u, p, mhat, mode=HESS_FULL):
        """H mhat per Eq. eq:incrementals3:

        (H mhat)_v = (R mhat)_v + sum_{T∋v} (c_T/3) |T| [grad u . grad phat + grad uhat . grad p]
                     + sum_{T∋v} (c_T/9) (sum_{w in T} mhat_w) |T| grad u . grad p.
        MISFIT omits R mhat; Gauss-Newton keeps only the grad u . grad phat term
        (with phat from the Gauss-Newton incremental adjoint).
        """
        gn = mode in (HESS_GN_FULL, HESS_GN_MISFIT)
        with_prior = mode in (HESS_FULL, HESS_GN_FULL)
        mhat = np.asarray(mhat, dtype=float)
        cT = self.coefficient(m)
        uh = self.inc_forward(m, u, mhat)
        ph = self.inc_adjoint(m, p, mhat, uh, gauss_newton=gn)
        per_tri = cT / 3.0 * self._tri_forms(u, ph)
        if not gn:
            per_tri = per_tri + cT / 3.0 * self._tri_forms(uh, p)
            msum = mhat[self.mesh.tris].sum(axis=1)
            per_tri = per_tri + cT / 9.0 * msum * self._tri_forms(u, p)
        out = self._vertex_sum(per_tri)
        if with_prior:
            out = out + self.R_apply(mhat)
        return out


def make_instance(cfg: dict, seed: int, eta_truth: np.ndarray, obs_xy: np.ndarray,
                  xi: np.ndarray, beta: float | None = None) -> tuple[Problem, np.ndarray, np.ndarray]:
    """Synthetic instance: m_true ~ N(m_pr, R^{-1}); d = B u(m_true) + sigma xi with
    sigma = 1% of max|u_true| (Sec. 5.1 observation model).

    Returns (problem, m_true, u_true).  The random inputs come from ``synth``.
    cfg["theta"] = (theta1, theta2, alpha), if present, gives the prior's
    anisotropic tensor (mesh.anisotropic_theta).
    """
    Theta = msh.anisotropic_theta(*cfg["theta"]) if cfg.get("theta") else None
    prob = Problem(cfg["N"], cfg["gamma"], cfg["delta"], cfg["m_prior"], beta=beta, Theta=Theta,
                   obs_xy=obs_xy, state_degree=cfg.get("state_degree", 1))
    m_true = prob.prior_sample(eta_truth)
    u_true = prob.forward(m_true)
    sigma = 0.01 * float(np.max(np.abs(u_true)))
    prob.sigma = sigma
    prob.d = prob.B @ u_true + sigma * xi
    prob._fact_m = None
    return prob, m_true, u_true
