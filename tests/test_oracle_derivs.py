"""Pins of the oracle's gradient and Hessian action.

Finite differences of the cost and of the gradient (the paper's own check,
Sec. 1), symmetry of the Hessian, and brute-force dense Hessians built from
second differences of the cost functional alone on a tiny mesh; each for the
P1 state and for the P2 state of the paper's Sec. 5.1 pairing (deg = 2).
"""
import numpy as np
import pytest

import synth
from oracle import model


DEGREES = pytest.mark.parametrize("deg", [1, 2])


def _instance(N=8, q=12, seed=1909, deg=1):
    cfg = dict(N=N, q=q, gamma=0.1, delta=0.5, m_prior=-2.0, state_degree=deg)
    prob, mt, _ = model.make_instance(cfg, seed, synth.white_noise(N, seed=seed)[0],
                                      synth.obs_points(q, seed=seed), synth.obs_noise(q, seed=seed))
    m = prob.m_pr + 0.4 * synth.smooth_field(N, seed=seed)
    return prob, m


def _fd_rates(errs):
    return [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]


@DEGREES
def test_gradient_central_differences_second_order(deg):
    prob, m = _instance(deg=deg)
    u = prob.forward(m)
    g = prob.gradient(m, u, prob.adjoint(m, u))
    dm = synth.test_vectors(prob.n, 1)[0]
    gd = g @ dm
    errs = []
    for eps in (1e-2, 1e-3):
        Jp = prob.cost(m + eps * dm)[0]
        Jm = prob.cost(m - eps * dm)[0]
        errs.append(abs((Jp - Jm) / (2 * eps) - gd) / abs(gd))
    assert errs[1] < 1e-6
    assert 50 < errs[0] / errs[1] < 200   # O(eps^2)


@pytest.mark.parametrize("mode", [model.HESS_FULL, model.HESS_MISFIT])
@DEGREES
def test_hessian_central_differences_of_gradient(mode, deg):
    prob, m = _instance(deg=deg)
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    dm = synth.test_vectors(prob.n, 1, stream=9)[0]
    H = prob.hessian_apply(m, u, p, dm, mode)
    errs = []
    for eps in (1e-2, 1e-3):
        gs = []
        for sgn in (1, -1):
            ms = m + sgn * eps * dm
            us = prob.forward(ms)
            g = prob.gradient(ms, us, prob.adjoint(ms, us))
            if mode == model.HESS_MISFIT:
                g = g - prob.R_apply(ms - prob.m_pr)
            gs.append(g)
        fd = (gs[0] - gs[1]) / (2 * eps)
        errs.append(np.linalg.norm(fd - H) / np.linalg.norm(H))
    assert errs[1] < 1e-6
    assert 50 < errs[0] / errs[1] < 200


@pytest.mark.parametrize("mode", [model.HESS_FULL, model.HESS_MISFIT,
                                  model.HESS_GN_FULL, model.HESS_GN_MISFIT])
@DEGREES
def test_hessian_symmetry(mode, deg):
    prob, m = _instance(deg=deg)
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    v1, v2 = synth.test_vectors(prob.n, 2, stream=10)
    a = v1 @ prob.hessian_apply(m, u, p, v2, mode)
    b = v2 @ prob.hessian_apply(m, u, p, v1, mode)
    assert abs(a - b) <= 1e-11 * max(abs(a), 1.0)


@DEGREES
def test_misfit_hessian_matches_second_differences_of_cost(deg):
    """Dense misfit Hessian from mixed second differences of the misfit term alone (N = 3)."""
    prob, m = _instance(N=3, q=6, deg=deg)
    n = prob.n
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    Hcols = np.column_stack([prob.hessian_apply(m, u, p, np.eye(n)[j], model.HESS_MISFIT)
                             for j in range(n)])
    eps = 1e-3
    E = np.eye(n) * eps

    def phi(x):
        return prob.misfit(prob.forward(x))

    Hfd = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            v = (phi(m + E[i] + E[j]) - phi(m + E[i] - E[j])
                 - phi(m - E[i] + E[j]) + phi(m - E[i] - E[j])) / (4 * eps * eps)
            Hfd[i, j] = Hfd[j, i] = v
    assert np.linalg.norm(Hfd - Hcols) / np.linalg.norm(Hcols) < 1e-5


@DEGREES
def test_gauss_newton_matches_brute_force_jacobian(deg):
    """GN misfit Hessian = J^T J / sigma^2 with J the FD Jacobian of m -> B u(m) (N = 4)."""
    prob, m = _instance(N=4, q=9, deg=deg)
    n = prob.n
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    eps = 1e-5
    J = np.column_stack([(prob.B @ prob.forward(m + eps * e) - prob.B @ prob.forward(m - eps * e)) / (2 * eps)
                         for e in np.eye(n)])
    Hgn = J.T @ J / prob.sigma ** 2
    Hcols = np.column_stack([prob.hessian_apply(m, u, p, e, model.HESS_GN_MISFIT) for e in np.eye(n)])
    assert np.linalg.norm(Hgn - Hcols) / np.linalg.norm(Hcols) < 1e-8
    Hfull = np.column_stack([prob.hessian_apply(m, u, p, e, model.HESS_GN_FULL) for e in np.eye(n)])
    Rd = np.column_stack([prob.R_apply(e) for e in np.eye(n)])
    assert np.linalg.norm(Hfull - Hcols - Rd) / np.linalg.norm(Hfull) < 1e-12


@DEGREES
def test_incremental_forward_is_derivative_of_state(deg):
    prob, m = _instance(deg=deg)
    u = prob.forward(m)
    dm = synth.test_vectors(prob.n, 1, stream=12)[0]
    uh = prob.inc_forward(m, u, dm)
    eps = 1e-4
    fd = (prob.forward(m + eps * dm) - prob.forward(m - eps * dm)) / (2 * eps)
    assert np.linalg.norm(fd - uh) / np.linalg.norm(uh) < 1e-7
    assert np.all(uh[~prob.free] == 0.0)
