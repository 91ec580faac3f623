"""GPU parity of the quadratic (P2) state (the state discretization of the
paper's Poisson experiment, Sec. 5.1) against the FP64 oracle, through the
C ABI.

* operator: A_2 x on the free rows within 1e-12 (N = 8, 16);
* solves (FP64 PCG with the two-level P2/P1 preconditioner) within 1e-8 for
  one and nine columns; the iteration counts are printed and bounded (the
  cycle is mesh-independent: at most 25 iterations to 1e-10 at N = 8 ... 64);
* forward, cost, adjoint and gradient within 1e-8 (cost 1e-10) at N = 16, 32,
  in the 2-norm and entry by entry (relative to the largest entry);
* incremental forward/adjoint and the Hessian action in all four modes
  within 1e-8, one and five columns, at N = 16;
* rejections: a P2 problem in a batch, in flexible CG and in the pair
  harvest (HINV_EINVAL); state vectors shorter than (2N+1)^2 (ValueError).
"""
import numpy as np
import pytest

import synth
from cases import col_maxabs, col_rel, instance, rel
from oracle import model

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


def p2_instance(N, q):
    return instance(N, q, state_degree=2)


def gpu_problem(ctx, prob, obs, precision=hv.PREC_AUTO):
    return hv.Problem(ctx, prob.N, prob.gamma, prob.delta, obs_xy=obs, d_obs=prob.d, sigma=prob.sigma,
                      beta=prob.beta, precision=precision, rtol=1e-10, state_degree=2)


def lin_point(prob, N):
    m = prob.m_pr + 0.4 * synth.smooth_field(N)
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    return m, u, p


def free_vectors(prob, nc, seed):
    X = synth.test_vectors(prob.ns, nc, seed=seed)
    X[:, ~prob.free] = 0.0
    return X


@pytest.mark.parametrize("N", [8, 16])
def test_p2_operator_and_solves(ctx, N):
    print(f"[gpu-p2] operator and solves N={N}", flush=True)
    prob, _, obs = p2_instance(N, 30)
    m, u, p = lin_point(prob, N)
    gp = gpu_problem(ctx, prob, obs)
    assert gp.ns == (2 * N + 1) ** 2
    gp.linearize(dev(m), dev(u), dev(p))
    A = prob.stiffness(m)
    f = prob.free
    X = free_vectors(prob, 3, 80)
    Y = dev(np.zeros_like(X))
    gp.state_apply(dev(X), Y)
    ref = np.array([np.where(f, A @ x, 0.0) for x in X])
    ea = col_rel(host(Y), ref)
    for nc in (1, 9):
        B = free_vectors(prob, nc, 81 + nc)
        Xs = dev(np.zeros_like(B))
        info = gp.state_solve(dev(B), Xs)
        sol = np.zeros_like(B)
        for c in range(nc):
            sol[c, f] = prob._solve_free(m, B[c, f])
        es = col_rel(host(Xs), sol)
        its = info["iterations"]
        print(f"[gpu-p2] N={N} nc={nc}: A x {ea:.1e}, solve {es:.1e}, {its} PCG iterations, "
              f"relres {info['max_relres']:.1e}", flush=True)
        assert info["rc"] == hv.HINV_OK and info["max_relres"] <= 1e-10, info
        assert es <= 1e-8 and its <= 25
    assert ea <= 1e-12


@pytest.mark.parametrize("N", [16, 32])
def test_p2_forward_cost_gradient(ctx, N):
    print(f"[gpu-p2] forward / gradient N={N}", flush=True)
    prob, _, obs = p2_instance(N, 60)
    gp = gpu_problem(ctx, prob, obs)
    m = prob.m_pr + 0.4 * synth.smooth_field(N)
    md, ud, pd, gd = dev(m), dev(np.zeros(prob.ns)), dev(np.zeros(prob.ns)), dev(np.zeros(prob.n))
    info = gp.forward(md, ud)
    assert info["rc"] == hv.HINV_OK, info
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    g = prob.gradient(m, u, p)
    mis, reg = gp.cost(md, ud)
    _, mis_o, reg_o = prob.cost(m, u)
    gp.gradient(md, ud, pd, gd)
    eu, ep, eg = (max(rel(host(a), b), col_maxabs(host(a), b)) for a, b in ((ud, u), (pd, p), (gd, g)))
    print(f"[gpu-p2] u {eu:.1e} p {ep:.1e} g {eg:.1e} misfit {abs(mis - mis_o) / mis_o:.1e}", flush=True)
    assert eu <= 1e-8 and ep <= 1e-8 and eg <= 1e-8
    assert abs(mis - mis_o) <= 1e-8 * mis_o and abs(reg - reg_o) <= 1e-10 * reg_o


@pytest.mark.parametrize("nc", [1, 5])
def test_p2_incremental_and_hessian(ctx, nc):
    N = 16
    print(f"[gpu-p2] Hessian actions N={N} nc={nc}", flush=True)
    prob, _, obs = p2_instance(N, 60)
    m, u, p = lin_point(prob, N)
    gp = gpu_problem(ctx, prob, obs)
    gp.linearize(dev(m), dev(u), dev(p))
    mh = synth.test_vectors(prob.n, nc, seed=84)
    uh = dev(np.zeros((nc, prob.ns)))
    gp.inc_forward(dev(mh), uh)
    uh_o = np.array([prob.inc_forward(m, u, v) for v in mh])
    e_uh = col_rel(host(uh), uh_o)
    ph = dev(np.zeros((nc, prob.ns)))
    for gn in (False, True):
        gp.inc_adjoint(dev(mh), dev(uh_o), ph, gauss_newton=gn)
        ph_o = np.array([prob.inc_adjoint(m, p, v, w, gauss_newton=gn) for v, w in zip(mh, uh_o)])
        assert col_rel(host(ph), ph_o) <= 1e-8
    errs = {}
    for mode in (hv.HESS_FULL, hv.HESS_MISFIT, hv.HESS_GN_FULL, hv.HESS_GN_MISFIT):
        out = dev(np.zeros((nc, prob.n)))
        info = gp.hessian_apply(mode, dev(mh), out)
        assert info["rc"] == hv.HINV_OK, info
        ref = np.array([prob.hessian_apply(m, u, p, v, mode) for v in mh])
        errs[mode] = max(col_rel(host(out), ref), col_maxabs(host(out), ref))
    print(f"[gpu-p2] uhat {e_uh:.1e}, H modes {[f'{e:.1e}' for e in errs.values()]}", flush=True)
    assert e_uh <= 1e-8 and max(errs.values()) <= 1e-8


def test_p2_rejections(ctx):
    prob, _, obs = p2_instance(8, 20)
    gp = gpu_problem(ctx, prob, obs)
    with pytest.raises(hv.HinvError) as e:
        hv.Batch(ctx, [gp])
    assert e.value.code == hv.HINV_EINVAL
    m, u, p = lin_point(prob, 8)
    gp.linearize(dev(m), dev(u), dev(p))
    b = dev(np.zeros(prob.ns))
    with pytest.raises(hv.HinvError) as e:
        gp.state_solve_fcg(b, dev(np.zeros(prob.ns)))
    assert e.value.code == hv.HINV_EINVAL
    with pytest.raises(ValueError):
        gp.forward(dev(m), dev(np.zeros(prob.n)))   # a P1-sized state vector
