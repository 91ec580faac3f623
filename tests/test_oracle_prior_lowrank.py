"""Pins of the oracle's prior, eigensolver, posterior sampling and Newton-CG.

Exact identities of the rectangular factor (Appendix C), closed forms of the
prior operator, the statistics of prior draws, Algorithm 2 with as many probe
vectors as unknowns against a dense generalized eigensolver, the covariance
identities of the posterior sample (Sec. 4.3.2) and the Sherman-Morrison-
Woodbury form (Eq. eq:sm), and the Newton-CG MAP point against an independent
quasi-Newton minimizer.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.optimize as sopt

import synth
from oracle import lowrank, model, newton
from oracle import mesh as msh


def _dense(apply, n):
    return np.column_stack([apply(e) for e in np.eye(n)])


def test_prior_operator_closed_forms():
    prob = model.Problem(6, 0.1, 0.5, beta=0.0)
    one = np.ones(prob.n)
    # K 1 = 0, so K_A 1 = delta M 1 when beta = 0
    np.testing.assert_allclose(prob.KA @ one, 0.5 * (prob.M @ one), atol=1e-14)
    prob2 = model.Problem(6, 0.1, 0.5)
    # 1^T K_A 1 = delta * area + beta * perimeter
    assert abs(one @ (prob2.KA @ one) - (0.5 + 4 * prob2.beta)) < 1e-12
    R = _dense(prob2.R_apply, prob2.n)
    np.testing.assert_allclose(R, R.T, atol=1e-12 * np.abs(R).max())
    assert np.linalg.eigvalsh(0.5 * (R + R.T)).min() > 0
    x = synth.test_vectors(prob2.n, 1)[0]
    np.testing.assert_allclose(prob2.R_apply(prob2.R_solve(x)), x, rtol=1e-9, atol=1e-9)


def test_prior_sample_covariance_converges_to_R_inverse():
    prob = model.Problem(4, 0.1, 0.5)
    ns = 20000
    eta = synth.white_noise(4, ns, stream=synth.STREAM_TEST)
    X = np.array([prob.prior_sample(e) for e in eta]) - prob.m_pr
    C = X.T @ X / ns
    Rinv = _dense(prob.R_solve, prob.n)
    err = np.linalg.norm(C - Rinv) / np.linalg.norm(Rinv)
    assert err < 4.0 / np.sqrt(ns) * 3, err   # O(1/sqrt(ns)) statistical error
    assert err > 1e-4                          # genuinely random


def _tiny_problem(N=4, q=8):
    cfg = dict(N=N, q=q, gamma=0.1, delta=0.5, m_prior=-2.0)
    prob, mt, _ = model.make_instance(cfg, 1909, synth.white_noise(N)[0], synth.obs_points(q),
                                      synth.obs_noise(q))
    m = prob.m_pr + 0.3 * synth.smooth_field(N)
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    return prob, m, u, p


def test_pre_chol_qr_invariants():
    prob, m, u, p = _tiny_problem()
    Y = synth.test_vectors(prob.n, 7).T
    Q, Qbar, Rf = lowrank.pre_chol_qr(Y, prob.R_apply)
    Rd = _dense(prob.R_apply, prob.n)
    np.testing.assert_allclose(Q.T @ Rd @ Q, np.eye(7), atol=1e-10)
    np.testing.assert_allclose(Q @ Rf, Y, atol=1e-10 * np.abs(Y).max())
    np.testing.assert_allclose(Qbar, Rd @ Q, atol=1e-9 * np.abs(Qbar).max())


@pytest.mark.parametrize("gn", [False, True])
def test_double_pass_with_full_probe_set_is_exact(gn):
    """With as many probe vectors as unknowns, Algorithm 2 returns the exact
    generalized eigenvalues of (H_misfit, R) (dense LAPACK reference)."""
    prob, m, u, p = _tiny_problem()
    n = prob.n
    mode = model.HESS_GN_MISFIT if gn else model.HESS_MISFIT
    A = lambda v: prob.hessian_apply(m, u, p, v, mode)
    Om = synth.omega(n, n).T
    lam, V, ex = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om, k=10)
    Hd = _dense(A, n)
    Hd = 0.5 * (Hd + Hd.T)
    Rd = _dense(prob.R_apply, n)
    Rd = 0.5 * (Rd + Rd.T)
    ref = sla.eigh(Hd, Rd, eigvals_only=True)[::-1]
    np.testing.assert_allclose(lam, ref[:10], rtol=1e-8, atol=1e-10 * abs(ref[0]))
    np.testing.assert_allclose(V.T @ Rd @ V, np.eye(10), atol=1e-8)
    res = Hd @ V - Rd @ V * lam
    assert np.linalg.norm(res[:, :3]) < 1e-7 * abs(lam[0]) * np.linalg.norm(Rd @ V[:, :3])
    if gn:
        assert (ref[prob.B.shape[0]:] < 1e-8 * ref[0]).all()   # rank <= q


def test_symmetric_least_squares_solver():
    rng = np.random.default_rng(5)
    s = 6
    W = rng.standard_normal((s, s))
    X0 = rng.standard_normal((s, s))
    X0 = X0 + X0.T
    # consistent data: the symmetric X0 is recovered
    np.testing.assert_allclose(lowrank.symmetric_least_squares(W, X0 @ W), X0, atol=1e-11)
    # inconsistent data: the solution is symmetric and satisfies the normal
    # equations of the symmetric problem, X W W^T + W W^T X = Z W^T + W Z^T
    Z = rng.standard_normal((s, s))
    X = lowrank.symmetric_least_squares(W, Z)
    np.testing.assert_allclose(X, X.T, atol=1e-13)
    G = W @ W.T
    np.testing.assert_allclose(X @ G + G @ X, Z @ W.T + W @ Z.T, atol=1e-10)
    # and no symmetric perturbation lowers the residual
    r0 = np.linalg.norm(X @ W - Z)
    for _ in range(20):
        E = rng.standard_normal((s, s))
        assert np.linalg.norm((X + 1e-3 * (E + E.T)) @ W - Z) >= r0


@pytest.mark.parametrize("gn", [False, True])
def test_single_pass_with_full_probe_set_is_exact(gn):
    """Algorithm 3 with as many probe vectors as unknowns: Q spans the space,
    A = B Q T Q^T B holds exactly, and the eigenvalues are those of the dense
    generalized problem (H_misfit, R); the Saibaba-Lee-Kitanidis T as read
    agrees (in exact arithmetic both equal W^-T Omega^T A Omega W^-1)."""
    prob, m, u, p = _tiny_problem()
    n = prob.n
    mode = model.HESS_GN_MISFIT if gn else model.HESS_MISFIT
    A = lambda v: prob.hessian_apply(m, u, p, v, mode)
    Om = synth.omega(n, n).T
    lam, V, ex = lowrank.single_pass(A, prob.R_apply, prob.R_solve, Om, k=8)
    lam2, _, _ = lowrank.single_pass_slk(A, prob.R_apply, prob.R_solve, Om, k=8)
    Hd = _dense(A, n)
    Hd = 0.5 * (Hd + Hd.T)
    Rd = _dense(prob.R_apply, n)
    Rd = 0.5 * (Rd + Rd.T)
    ref = sla.eigh(Hd, Rd, eigvals_only=True)[::-1]
    np.testing.assert_allclose(lam, ref[:8], rtol=1e-6, atol=1e-9 * abs(ref[0]))
    np.testing.assert_allclose(lam2, ref[:8], rtol=1e-6, atol=1e-9 * abs(ref[0]))
    np.testing.assert_allclose(V.T @ Rd @ V, np.eye(8), atol=1e-8)
    # T is the symmetric least-squares solution: zero residual here
    W, Z, T = ex["W"], ex["Z"], ex["T"]
    assert np.linalg.norm(T @ W - Z) <= 1e-8 * np.linalg.norm(Z)


def test_single_pass_exact_for_low_rank_operator():
    """Gauss-Newton misfit Hessian with q observations has rank <= q; with
    s > q probe vectors the first pass captures its range and Algorithm 3 is
    exact for every nonzero eigenvalue, as is Algorithm 2."""
    prob, m, u, p = _tiny_problem(N=8, q=6)
    A = lambda v: prob.hessian_apply(m, u, p, v, model.HESS_GN_MISFIT)
    Om = synth.omega(prob.n, 10).T
    lam1, _, _ = lowrank.single_pass(A, prob.R_apply, prob.R_solve, Om, k=6)
    lam2, _, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om, k=6)
    Hd = _dense(A, prob.n)
    Rd = _dense(prob.R_apply, prob.n)
    ref = sla.eigh(0.5 * (Hd + Hd.T), 0.5 * (Rd + Rd.T), eigvals_only=True)[::-1][:6]
    np.testing.assert_allclose(lam2, ref, rtol=1e-7)
    np.testing.assert_allclose(lam1, ref, rtol=1e-6)


def test_prior_variance_exact_with_every_eigenpair():
    """Eq. eq:prior_mvar with rbar = n eigenpairs of R^-1 (Algorithm 2, B = I,
    l = 0) is the exact diagonal of R^-1; Eq. eq:post_mvar with every eigenpair
    of (H_misfit, R) is the exact diagonal of (H_misfit + R)^-1 (Eq. eq:sm with
    zero remainder); the stochastic estimator with the unit vectors as probes
    is exact too."""
    prob, m, u, p = _tiny_problem()
    n = prob.n
    Rd = _dense(prob.R_apply, n)
    Rd = 0.5 * (Rd + Rd.T)
    Rinv = np.linalg.inv(Rd)
    dg, mu = lowrank.prior_variance(prob.R_solve, synth.omega(n, n).T)
    np.testing.assert_allclose(dg, np.diag(Rinv), rtol=1e-8)
    assert np.all(np.diff(mu) <= 0) and mu[-1] > 0
    A = lambda v: prob.hessian_apply(m, u, p, v, model.HESS_GN_MISFIT)
    Hd = _dense(A, n)
    Hd = 0.5 * (Hd + Hd.T)
    lam, V = sla.eigh(Hd, Rd)
    post = lowrank.posterior_variance(np.diag(Rinv), V, lam)
    np.testing.assert_allclose(post, np.diag(np.linalg.inv(Hd + Rd)), rtol=1e-8)
    np.testing.assert_allclose(lowrank.stochastic_diagonal(prob.R_solve, np.eye(n)), np.diag(Rinv),
                               rtol=1e-10)


def test_prior_variance_converges_with_rank():
    """The truncated sum approaches diag(R^-1) as rbar grows (the eigenvalues of
    R^-1 decay fast: it is the discretization of a compact operator), and its
    eigenvalues mu_i are Ritz values of R^-1: below its largest eigenvalue."""
    prob, m, u, p = _tiny_problem(N=8)
    n = prob.n
    Rinv = np.linalg.inv(_dense(prob.R_apply, n))
    d = np.diag(Rinv)
    top = np.linalg.eigvalsh(0.5 * (Rinv + Rinv.T))[-1]
    errs = []
    for r in (5, 20, 60):
        dg, mu = lowrank.prior_variance(prob.R_solve, synth.omega(n, r).T)
        assert mu[0] <= top * (1 + 1e-10)
        errs.append(np.linalg.norm(dg - d) / np.linalg.norm(d))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-2, errs


def test_posterior_sample_covariance_identities():
    prob, m, u, p = _tiny_problem()
    n = prob.n
    A = lambda v: prob.hessian_apply(m, u, p, v, model.HESS_GN_MISFIT)
    Hd = _dense(A, n)
    Hd = 0.5 * (Hd + Hd.T)
    Rd = _dense(prob.R_apply, n)
    Rd = 0.5 * (Rd + Rd.T)
    lam, V = sla.eigh(Hd, Rd)
    lam, V = lam[::-1], V[:, ::-1]
    Rinv = np.linalg.inv(Rd)
    for r in (3, n):
        Vr, lr = V[:, :r], lam[:r]
        Map = np.column_stack([lowrank.posterior_sample_update(e, Vr, lr, prob.R_apply) for e in np.eye(n)])
        cov = Map @ Rinv @ Map.T
        D = lr / (1.0 + lr)
        np.testing.assert_allclose(cov, Rinv - (Vr * D) @ Vr.T, atol=1e-9 * np.abs(Rinv).max())
    # full rank: SMW with zero remainder (Eq. eq:sm)
    np.testing.assert_allclose(Rinv - (V * (lam / (1 + lam))) @ V.T, np.linalg.inv(Hd + Rd),
                               atol=1e-9 * np.abs(Rinv).max())
    with pytest.raises(ValueError):
        lowrank.posterior_sample_update(np.ones(n), V[:, :1], np.array([-1.5]), prob.R_apply)


def test_newton_cg_map_matches_quasi_newton_minimizer():
    N, q = 8, 20
    cfg = dict(N=N, q=q, gamma=0.1, delta=0.5, m_prior=-2.0)
    prob, mt, _ = model.make_instance(cfg, 1909, synth.white_noise(N)[0], synth.obs_points(q),
                                      synth.obs_noise(q))
    m_map, info = newton.newton_cg(prob, rel_tol=1e-9)
    assert info["converged"]
    gn = info["gnorm"]
    assert gn[-1] <= 1e-9 * gn[0]

    def fg(x):
        u = prob.forward(x)
        J = prob.cost(x, u)[0]
        return J, prob.gradient(x, u, prob.adjoint(x, u))

    res = sopt.minimize(fg, prob.m_pr.copy(), jac=True, method="L-BFGS-B",
                        options=dict(maxiter=20000, ftol=1e-15, gtol=1e-11 * gn[0], maxcor=50))
    Rd = _dense(prob.R_apply, prob.n)
    d = m_map - res.x
    rel = np.sqrt(d @ Rd @ d) / np.sqrt((m_map - prob.m_pr) @ Rd @ (m_map - prob.m_pr))
    assert rel < 1e-6, rel
