"""The paper's own Poisson setup (Sec. 5.1) on the GPU against the oracle: a
quadratic (P2) state with a linear parameter on 64 x 64 cells (16 641 state
and 4 225 parameter unknowns), the anisotropic prior
-gamma div(Theta grad m) + delta m with theta = (2, 0.5), alpha = pi/4 (Theta
as read: the s.p.d. tensor with those eigenvalues and directions), 50
observations in [0.1, 0.9] x [0.1, 0.5].

* prior R x, R^-1 x and prior draws with Theta: 1e-10 (apply) and 1e-8
  (solves) relative per column at N = 16 and 64;
* the full Hessian action (which contains R) at N = 32: 1e-8;
* MAP point (Alg. 1) within 1e-8 in the R-norm, eigenvalues of the
  Gauss-Newton misfit Hessian at the oracle's MAP point within 1e-8 lambda_1,
  with the section's r = 30 and l = 20 (s = 50 = q probe vectors), and with
  l = 40 (s = 70 > q: the Gauss-Newton block Y = R^-1 H Omega has rank <= q,
  qr(Y) keeps its numerical range);
  the spectrum is printed and compared with Fig. 7 qualitatively: it decays
  fast, and fewer eigenvalues exceed 0.07 than there are observations;
* pointwise variance (Sec. 4.4, the Fig. 8 analog) at the MAP point: the
  prior variance from r = 300 eigenpairs of R^-1 and the posterior variance
  with the Gauss-Newton eigenpairs, each within 1e-8 of the oracle's; the
  data lower the variance most inside the observation box;
* a tensor whose off-diagonal has the wrong sign for this mesh is rejected.
"""
import numpy as np
import pytest

import synth
from cases import col_rel, rel
from oracle import lowrank, model, newton
from oracle import mesh as msh

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hv = pytest.importorskip("paper_1909_03948_amd.hinv")

CFG = synth.WORKLOADS["poisson64_paper"]
THETA = CFG["theta"]


@pytest.fixture(scope="module")
def ctx():
    return hv.Context(0)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def paper_instance(N):
    cfg = dict(CFG, N=N)
    q = cfg["q"]
    obs = synth.obs_points(q, box=cfg["obs_box"])
    prob, m_true, _ = model.make_instance(cfg, synth.MASTER_SEED, synth.white_noise(N)[0], obs,
                                          synth.obs_noise(q))
    return prob, obs


def gpu_problem(ctx, prob, obs, precision=hv.PREC_AUTO, theta=THETA):
    return hv.Problem(ctx, prob.N, prob.gamma, prob.delta, obs_xy=obs, d_obs=prob.d, sigma=prob.sigma,
                      m_prior=prob.m_pr[0], beta=prob.beta, precision=precision, rtol=1e-10, theta=theta,
                      state_degree=CFG["state_degree"])


@pytest.mark.parametrize("N", [16, 64])
def test_anisotropic_prior_apply_solve_sample(ctx, N):
    print(f"[gpu-paper] anisotropic prior N={N}", flush=True)
    prob, obs = paper_instance(N)
    gp = gpu_problem(ctx, prob, obs)
    X = synth.test_vectors(prob.n, 9, seed=70)
    Y = dev(np.zeros_like(X))
    gp.prior_apply(dev(X), Y)
    ea = col_rel(host(Y), np.array([prob.R_apply(x) for x in X]))
    gp.prior_solve(dev(X), Y)
    es = col_rel(host(Y), np.array([prob.R_solve(x) for x in X]))
    eta = synth.white_noise(N, 3, stream=synth.STREAM_POST)
    out = dev(np.zeros((3, prob.n)))
    gp.prior_sample(dev(eta), out)
    ep = col_rel(host(out), np.array([prob.prior_sample(e) for e in eta]))
    print(f"[gpu-paper] R x {ea:.2e}, R^-1 x {es:.2e}, prior draws {ep:.2e}", flush=True)
    assert ea <= 1e-10 and es <= 1e-8 and ep <= 1e-8


def test_full_hessian_with_anisotropic_prior(ctx):
    prob, obs = paper_instance(32)
    m = prob.m_pr + 0.4 * synth.smooth_field(32)
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    gp = gpu_problem(ctx, prob, obs)
    gp.linearize(dev(m), dev(u), dev(p))
    mh = synth.test_vectors(prob.n, 3, seed=71)
    out = dev(np.zeros((3, prob.n)))
    assert prob.ns == gp.ns == 65 ** 2
    gp.hessian_apply(hv.HESS_FULL, dev(mh), out)
    ref = np.array([prob.hessian_apply(m, u, p, v, model.HESS_FULL) for v in mh])
    assert col_rel(host(out), ref) <= 1e-8


def test_paper_setup_map_and_spectrum(ctx):
    prob, obs = paper_instance(64)
    m_o, info_o = newton.newton_cg(prob, rel_tol=1e-11)
    gp = gpu_problem(ctx, prob, obs)
    md = dev(np.zeros(prob.n))
    info = gp.map_newton(md, rel_tol=1e-11)
    assert info["rc"] in (hv.HINV_OK, hv.HINV_ESTATE) and info["gnorm"][-1] <= 1e-9 * info["gnorm"][0], info
    d = host(md) - m_o
    dm = m_o - prob.m_pr
    err = np.sqrt(d @ prob.R_apply(d)) / np.sqrt(dm @ prob.R_apply(dm))
    print(f"[gpu-paper] MAP: {info['iterations']} Newton iterations, R-norm rel diff {err:.2e}", flush=True)
    assert err <= 1e-8
    u = prob.forward(m_o)
    p = prob.adjoint(m_o, u)
    k, s = CFG["k"], CFG["k"] + CFG["p"]
    Om = synth.omega(prob.n, s)
    A = lambda v: prob.hessian_apply(m_o, u, p, v, model.HESS_GN_MISFIT)
    lam_o, _, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om.T, k)
    gp.linearize(dev(m_o), dev(u), dev(p))
    V = dev(np.zeros((k, prob.n)))
    lam, _ = gp.lowrank_eig(dev(Om), k, V, mode=hv.HESS_GN_MISFIT)
    e = np.max(np.abs(lam - lam_o)) / lam_o[0]
    above = int(np.sum(lam > 0.07))
    print(f"[gpu-paper] eigenvalues: max |dlambda|/lambda_1 {e:.2e}; {above} above 0.07, "
          f"{int(np.sum(lam > 1))} above 1 (q = {CFG['q']})", flush=True)
    print("[gpu-paper] lambda_1..30:", np.array2string(lam, precision=3), flush=True)
    assert e <= 1e-8
    assert above < CFG["q"] and lam[0] / lam[-1] > 100
    # more probes than observations: a rank-deficient probe block
    s70 = k + 40
    Om70 = synth.omega(prob.n, s70)
    lam70_o, _, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om70.T, k)
    V70 = dev(np.zeros((k, prob.n)))
    lam70, info = gp.lowrank_eig(dev(Om70), k, V70, mode=hv.HESS_GN_MISFIT)
    assert info["rc"] == 0, info
    e70 = np.max(np.abs(lam70 - lam70_o)) / lam70_o[0]
    print(f"[gpu-paper] s = {s70} > q: max |dlambda|/lambda_1 {e70:.2e}; against s = {s}: "
          f"{np.max(np.abs(lam70 - lam)) / lam[0]:.2e}", flush=True)
    assert e70 <= 1e-8
    # pointwise variance at the MAP point (Fig. 8 analog)
    rbar = 300
    Omv = synth.omega(prob.n, rbar, seed=synth.MASTER_SEED + 7)
    pd_o, _ = lowrank.prior_variance(prob.R_solve, Omv.T)
    pdg = dev(np.zeros(prob.n))
    mu, info = gp.prior_variance(dev(Omv), pdg)
    assert info["rc"] == 0, info
    ep = rel(host(pdg), pd_o)
    _, V_o, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om.T, k)
    post_o = lowrank.posterior_variance(pd_o, V_o, lam_o)
    post = dev(np.zeros(prob.n))
    gp.posterior_variance(pdg, lam, V, post)
    eq = rel(host(post), post_o)
    ratio = host(post) / host(pdg)
    xy = np.array([(i / 64, j / 64) for j in range(65) for i in range(65)])
    box = (xy[:, 0] >= 0.1) & (xy[:, 0] <= 0.9) & (xy[:, 1] >= 0.1) & (xy[:, 1] <= 0.5)
    print(f"[gpu-paper] variance (rbar = {rbar}): prior {ep:.1e}, posterior {eq:.1e} from the oracle; "
          f"max prior variance {host(pdg).max():.3e}; mean posterior/prior inside the box "
          f"{ratio[box].mean():.3f}, outside {ratio[~box].mean():.3f}", flush=True)
    assert ep <= 1e-8 and eq <= 1e-8
    assert ratio[box].mean() < ratio[~box].mean() and np.all(ratio <= 1 + 1e-12)


def test_tensor_outside_the_mesh_condition_is_rejected(ctx):
    prob, obs = paper_instance(16)
    with pytest.raises(hv.HinvError) as e:
        gpu_problem(ctx, prob, obs, theta=(2.0, 0.5, -np.pi / 4))
    assert e.value.code == hv.HINV_EINVAL
    np.testing.assert_allclose(msh.anisotropic_theta(*THETA), [[1.25, 0.75], [0.75, 1.25]], atol=1e-14)
