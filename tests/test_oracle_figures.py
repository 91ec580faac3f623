"""Analogs of the paper's accuracy comparisons, computed with the oracle on the
32 x 32 workload (n = 1 089; the paper's Poisson example has n = 4 225):

* Fig. 2: the first 30 generalized eigenvalues of the Gauss-Newton data-misfit
  Hessian at the MAP point from a dense eigensolver (exact), Algorithm 2
  (double pass), Algorithm 3 (single pass) and the single-pass T of Saibaba,
  Lee & Kitanidis (as read, see oracle/lowrank.py), for oversampling
  l = 5, 10, 20.
* Fig. 4: the L2 relative error of the prior's pointwise variance from the
  randomized eigendecomposition of R^-1 (Eq. eq:prior_mvar) against the
  stochastic estimator (Eq. eq:stoc_diag_estimator) for a given number of
  R^-1 applications (a), and at fixed rank over mesh sizes (b).

Both print their tables (pytest -s); the assertions hold the qualitative
findings: the double pass is at least as accurate as the single pass, the
errors fall with l, the eigendecomposition estimator beats the stochastic
one at equal cost, and its error does not grow with the mesh.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from cases import instance
from oracle import lowrank, model, newton


def _dense(apply, n):
    A = np.column_stack([apply(e) for e in np.eye(n)])
    return 0.5 * (A + A.T)


@pytest.mark.slow
def test_fig2_analog_single_vs_double_pass():
    prob, _, _ = instance(32, 100)
    m, info = newton.newton_cg(prob, rel_tol=1e-9)
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    A = lambda v: prob.hessian_apply(m, u, p, v, model.HESS_GN_MISFIT)
    n, r = prob.n, 30
    exact = sla.eigh(_dense(A, n), _dense(prob.R_apply, n), eigvals_only=True)[::-1][:r]
    rows = {}
    for l in (5, 10, 20):
        Om = synth.omega(n, r + l, seed=1909 + l).T
        res = {}
        for name, fn in (("double", lowrank.double_pass), ("single", lowrank.single_pass),
                         ("slk", lowrank.single_pass_slk)):
            lam, _, _ = fn(A, prob.R_apply, prob.R_solve, Om, r)
            res[name] = np.abs(lam - exact) / exact
        rows[l] = res
        print(f"[fig2] l={l:2d}  max rel err over the first {r}: double {res['double'].max():.2e}  "
              f"single (Alg. 3) {res['single'].max():.2e}  SLK {res['slk'].max():.2e}; "
              f"lambda_10: {res['double'][9]:.1e} / {res['single'][9]:.1e} / {res['slk'][9]:.1e}")
    print("[fig2] exact lambda_1, lambda_10, lambda_30:", exact[0], exact[9], exact[29])
    for l in (5, 10, 20):
        assert rows[l]["double"].max() <= rows[l]["single"].max()
        assert np.median(rows[l]["double"]) <= np.median(rows[l]["single"])
    assert rows[20]["double"].max() < rows[5]["double"].max()
    assert rows[20]["single"].max() < rows[5]["single"].max()
    # the double pass captures the leading eigenvalues at every l
    for l in (5, 10, 20):
        assert rows[l]["double"][:5].max() < 1e-3
    # Algorithm 3 and the SLK T as read are one matrix in exact arithmetic
    # (W^T R = Omega^T A Omega makes R W^-1 symmetric, so the symmetric
    # least-squares problem has the zero-residual solution R W^-1 =
    # W^-T Omega^T Ybar W^-1): they agree to rounding, so the gap the paper
    # plots is not reproduced under this reading
    for l in (5, 10, 20):
        assert np.max(np.abs(rows[l]["single"] - rows[l]["slk"])) < 1e-6


def _mnorm(M, v):
    return float(np.sqrt(v @ (M @ v)))


@pytest.mark.slow
def test_fig4_analog_prior_variance_estimators():
    # (a) error against the number of R^-1 applications at N = 32
    prob = model.Problem(32, 0.1, 0.5)
    n = prob.n
    Rd = _dense(prob.R_apply, n)
    exact = np.diag(np.linalg.inv(Rd))
    M = prob.M
    nex = _mnorm(M, exact)
    rng = np.random.default_rng(4)
    print("[fig4a] applies  randomized-eig  stochastic")
    errs = []
    for applies in (20, 40, 80, 160, 320):
        dg, _ = lowrank.prior_variance(prob.R_solve, synth.omega(n, applies // 2, seed=applies).T)
        Z = rng.choice([-1.0, 1.0], size=(n, applies))
        st = lowrank.stochastic_diagonal(prob.R_solve, Z)
        e1, e2 = _mnorm(M, dg - exact) / nex, _mnorm(M, st - exact) / nex
        errs.append((applies, e1, e2))
        print(f"[fig4a] {applies:7d}  {e1:.2e}        {e2:.2e}")
    for applies, e1, e2 in errs:
        if applies >= 40:
            assert e1 < e2, (applies, e1, e2)
    assert errs[-1][1] < errs[0][1]
    # (b) fixed rank rbar = 50 over mesh sizes: the error does not grow with n
    print("[fig4b] N   n      rel err (rbar = 50)")
    eb = []
    for N in (16, 32, 64):
        pr = model.Problem(N, 0.1, 0.5)
        d = np.diag(np.linalg.inv(_dense(pr.R_apply, pr.n)))
        dg, _ = lowrank.prior_variance(pr.R_solve, synth.omega(pr.n, 50, seed=N).T)
        e = _mnorm(pr.M, dg - d) / _mnorm(pr.M, d)
        eb.append(e)
        print(f"[fig4b] {N:3d} {pr.n:5d}  {e:.2e}")
    assert max(eb) < 2.0 * min(eb)
