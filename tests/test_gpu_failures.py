"""Failure behaviour of the C ABI, forced from the host (every kernel still
exits normally):

* an iteration limit of 1 per solve: HINV_ENOCONV, the outputs written (finite,
  nonzero) and info.status / info.max_relres set, for one column and a batch,
  in both solve precisions; the problem stays usable afterwards;
* a NaN in a right-hand side or in a Hessian direction: that column stops at
  once, the call returns HINV_ENOCONV with max_relres NaN, the other columns
  of the same call are solved to the oracle's bar, and the next call is clean;
* Newton-CG with no backtracking step allowed: the line search fails at the
  first iteration (HINV_ESTATE) and leaves the starting point; with one Newton
  iteration allowed it stops unconverged (HINV_ENOCONV).
"""
import math

import numpy as np
import pytest

import synth
from cases import instance, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hv = pytest.importorskip("paper_1909_03948_amd.hinv")


@pytest.fixture(scope="module")
def ctx():
    return hv.Context(0)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def lin32(ctx):
    prob, _, obs = instance(32, 100)
    m = prob.m_pr + 0.3 * synth.smooth_field(32)
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    return prob, obs, m, u, p


def gpu_problem(ctx, prob, obs, lin, precision):
    _, _, m, u, p = lin
    gp = hv.Problem(ctx, prob.N, prob.gamma, prob.delta, obs_xy=obs, d_obs=prob.d, sigma=prob.sigma,
                    beta=prob.beta, precision=precision, rtol=1e-10)
    gp.linearize(dev(m), dev(u), dev(p))
    return gp


def free_rhs(prob, nc, seed):
    b = synth.test_vectors(prob.n, nc, seed=seed)
    b[:, ~prob.free] = 0.0
    return b


@pytest.mark.parametrize("prec", [hv.PREC_FP64, hv.PREC_FP32_IR])
@pytest.mark.parametrize("nc", [1, 8])
def test_iteration_limit_reports_noconv_with_outputs_written(ctx, lin32, prec, nc):
    print(f"[gpu-fail] max_iter = 1, prec={prec}, nc={nc}", flush=True)
    prob, obs, *_ = lin32
    gp = gpu_problem(ctx, prob, obs, lin32, prec)
    gp.set_solver(prec, 1e-10, 1)
    b = free_rhs(prob, nc, 60)
    x = dev(np.zeros((nc, prob.n)))
    info = gp.state_solve(dev(b), x)
    assert info["rc"] == hv.HINV_ENOCONV and info["status"] == hv.HINV_ENOCONV, info
    assert info["max_relres"] > 1e-10 and math.isfinite(info["max_relres"]), info
    X = host(x)
    assert np.all(np.isfinite(X)) and np.all(np.abs(X).max(axis=1) > 0)
    mh = dev(synth.test_vectors(prob.n, nc, seed=61))
    out = dev(np.zeros((nc, prob.n)))
    info = gp.hessian_apply(hv.HESS_FULL, mh, out)
    assert info["rc"] == hv.HINV_ENOCONV, info
    assert np.all(np.isfinite(host(out)))
    # with the limit lifted the same problem solves to its tolerance
    gp.set_solver(prec, 1e-10, 0)
    info = gp.state_solve(dev(b), x)
    assert info["rc"] == hv.HINV_OK and info["max_relres"] <= 1e-10, info


@pytest.mark.parametrize("prec", [hv.PREC_FP64, hv.PREC_FP32_IR])
def test_nan_in_input_stops_its_column(ctx, lin32, prec):
    print(f"[gpu-fail] NaN input, prec={prec}", flush=True)
    prob, obs, m, u, p = lin32
    gp = gpu_problem(ctx, prob, obs, lin32, prec)
    nc = 8 if prec == hv.PREC_FP32_IR else 2
    b = free_rhs(prob, nc, 62)
    b[0, prob.n // 2] = np.nan
    x = dev(np.zeros((nc, prob.n)))
    info = gp.state_solve(dev(b), x)
    assert info["rc"] == hv.HINV_ENOCONV and math.isnan(info["max_relres"]), info
    X = host(x)
    f = prob.free
    for c in range(1, nc):
        ref = np.zeros(prob.n)
        ref[f] = prob._solve_free(m, b[c][f])
        assert rel(X[c], ref) <= 1e-8, c
    mh = synth.test_vectors(prob.n, nc, seed=63)
    mh[nc - 1, 3] = np.inf
    out = dev(np.zeros((nc, prob.n)))
    info = gp.hessian_apply(hv.HESS_MISFIT, dev(mh), out)
    assert info["rc"] == hv.HINV_ENOCONV and math.isnan(info["max_relres"]), info
    # the next call is clean
    info = gp.state_solve(dev(free_rhs(prob, nc, 64)), x)
    assert info["rc"] == hv.HINV_OK and info["max_relres"] <= 1e-10, info


def test_newton_line_search_failure_and_iteration_limit(ctx, lin32):
    prob, obs, *_ = lin32
    gp = hv.Problem(ctx, prob.N, prob.gamma, prob.delta, obs_xy=obs, d_obs=prob.d, sigma=prob.sigma,
                    beta=prob.beta, precision=hv.PREC_FP64, rtol=1e-10)
    md = dev(np.zeros(prob.n))
    info = gp.map_newton(md, rel_tol=1e-6, max_backtrack=0)
    print(f"[gpu-fail] max_backtrack = 0: rc {info['rc']}, iterations {info['iterations']}", flush=True)
    assert info["rc"] == hv.HINV_ESTATE and info["status"] == hv.HINV_ESTATE and not info["converged"]
    assert info["iterations"] == 1
    assert np.array_equal(host(md), prob.m_pr)
    info = gp.map_newton(md, rel_tol=1e-6, max_iter=1)
    assert info["rc"] == hv.HINV_ENOCONV and info["iterations"] == 1 and not info["converged"], info
    assert info["gnorm"][1] < info["gnorm"][0]
