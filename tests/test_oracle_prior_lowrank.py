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
