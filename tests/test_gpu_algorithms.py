"""GPU parity of the paper's algorithms against the FP64 oracle.

* MAP point (Alg. 1): the oracle's own gradient at the GPU's MAP point is
  <= 1e-8 |g_0|, and the two MAP points agree to <= 1e-8 in the R-norm
  relative to |m_map - m_pr|_R (both run Newton-CG to |g| <= 1e-11 |g_0| or
  to the floor where Armijo can no longer resolve the decrease of J).
* Eigenpairs (Alg. 2 + Alg. 4) at the oracle's MAP point with the same probe
  matrix: |lambda_gpu - lambda_orc| <= 1e-8 lambda_1 for all k, relative error
  <= 1e-8 for the leading eigenvalues (lambda >= 1e-2 lambda_1), eigenvectors
  R-orthonormal and equal up to sign for well-separated leading pairs.
* Posterior samples (Eq. eq:sample_post) with the same eta, V, Lambda: <= 1e-8.
"""
import numpy as np
import pytest

import synth
from cases import col_rel, instance, rel
from oracle import lowrank, model, newton

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


def gpu_problem(ctx, prob, obs, precision=hv.PREC_FP64):
    return hv.Problem(ctx, prob.N, prob.gamma, prob.delta, obs_xy=obs, d_obs=prob.d,
                      sigma=prob.sigma, m_prior=prob.m_pr[0], beta=prob.beta,
                      precision=precision, rtol=1e-10)


@pytest.fixture(scope="module")
def map32():
    prob, _, obs = instance(32, 100)
    m_map, info = newton.newton_cg(prob, rel_tol=1e-11)
    assert info["gnorm"][-1] <= 1e-10 * info["gnorm"][0], info
    return prob, obs, m_map


@pytest.mark.parametrize("prec", [hv.PREC_FP64, hv.PREC_FP32_IR])
def test_newton_map_point(ctx, map32, prec):
    print(f"[gpu] newton prec={prec}", flush=True)
    prob, obs, m_orc = map32
    gp = gpu_problem(ctx, prob, obs, prec)
    md = dev(np.zeros(prob.n))
    info = gp.map_newton(md, rel_tol=1e-11)
    # converged, or stopped by the line search at the floor of J's resolution
    assert info["rc"] in (hv.HINV_OK, hv.HINV_ESTATE), info
    assert info["gnorm"][-1] <= 1e-9 * info["gnorm"][0], info
    m_gpu = host(md)
    u = prob.forward(m_gpu)
    g = prob.gradient(m_gpu, u, prob.adjoint(m_gpu, u))
    g0 = info["gnorm"][0]
    assert np.linalg.norm(g) <= 1e-8 * g0
    d = m_gpu - m_orc
    dm = m_orc - prob.m_pr
    err = np.sqrt(d @ prob.R_apply(d)) / np.sqrt(dm @ prob.R_apply(dm))
    print(f"[gpu] MAP R-norm rel diff {err:.2e}, |g|/|g0| {info['gnorm'][-1] / g0:.2e}", flush=True)
    assert err <= 1e-8
    # Newton iterations are mesh-independent and few
    assert info["iterations"] <= 20


@pytest.mark.parametrize("mode", [hv.HESS_MISFIT, hv.HESS_GN_MISFIT])
@pytest.mark.parametrize("prec", [hv.PREC_FP64, hv.PREC_FP32_IR])
def test_double_pass_eigenpairs(ctx, map32, mode, prec):
    print(f"[gpu] double pass mode={mode} prec={prec}", flush=True)
    prob, obs, m = map32
    k, p = 50, 20
    s = k + p
    u = prob.forward(m)
    adj = prob.adjoint(m, u)
    Om = synth.omega(prob.n, s)
    A = lambda v: prob.hessian_apply(m, u, adj, v, mode)
    lam_o, V_o, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om.T, k)
    gp = gpu_problem(ctx, prob, obs, prec)
    gp.linearize(dev(m), dev(u), dev(adj))
    V = dev(np.zeros((k, prob.n)))
    lam, info = gp.lowrank_eig(dev(Om), k, V, mode=mode)
    assert info["rc"] == 0, info
    l1 = abs(lam_o[0])
    assert np.max(np.abs(lam - lam_o)) <= 1e-8 * l1
    lead = lam_o >= 1e-2 * l1
    assert np.max(np.abs(lam[lead] - lam_o[lead]) / np.abs(lam_o[lead])) <= 1e-8
    Vg = host(V).T
    RV = np.column_stack([prob.R_apply(v) for v in Vg.T])
    np.testing.assert_allclose(Vg.T @ RV, np.eye(k), atol=1e-8)
    gaps = np.abs(np.diff(lam_o))
    for i in range(5):
        sep = min(gaps[i], gaps[i - 1] if i > 0 else np.inf) / l1
        if sep > 1e-3:
            assert abs(abs(V_o[:, i] @ RV[:, i]) - 1.0) < 1e-6


@pytest.mark.parametrize("k,p", [(50, 21), (100, 9)])
def test_double_pass_odd_probe_counts(ctx, k, p):
    """Odd s = k + p on both sides of the size where the s x s factorizations
    leave LDS (s = 71 in LDS, s = 109 in global memory): the Jacobi sweeps
    then pair one index with a padding index every step."""
    s = k + p
    print(f"[gpu] double pass odd s={s}", flush=True)
    prob, m, obs = instance(32, 300)
    u = prob.forward(m)
    adj = prob.adjoint(m, u)
    Om = synth.omega(prob.n, s, seed=7)
    A = lambda v: prob.hessian_apply(m, u, adj, v, model.HESS_GN_MISFIT)
    lam_o, _, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om.T, k)
    gp = gpu_problem(ctx, prob, obs)
    gp.linearize(dev(m), dev(u), dev(adj))
    V = dev(np.zeros((k, prob.n)))
    lam, info = gp.lowrank_eig(dev(Om), k, V, mode=hv.HESS_GN_MISFIT)
    assert info["rc"] == 0, info
    l1 = abs(lam_o[0])
    assert np.max(np.abs(lam - lam_o)) <= 1e-8 * l1
    Vg = host(V).T
    RV = np.column_stack([prob.R_apply(v) for v in Vg.T])
    np.testing.assert_allclose(Vg.T @ RV, np.eye(k), atol=1e-8)


def test_double_pass_rank_deficient_probe_block(ctx):
    """A probe block with exactly zero columns has rank below s.  One problem:
    qr(Y) falls back to the leading directions of Y^T Y and the double pass
    returns the eigenpairs of the nonzero columns' span (equal to those from
    the probe block without the zero columns, 1e-8 lambda_1; V R-orthonormal);
    with fewer directions than k it reports HINV_EBREAK.  A batch whose member
    has such a block reports HINV_EBREAK (its Cholesky QR has no fallback);
    the problems stay usable."""
    prob, m, obs = instance(16, 40)
    u = prob.forward(m)
    adj = prob.adjoint(m, u)
    gps = [gpu_problem(ctx, prob, obs) for _ in range(2)]
    for gp in gps:
        gp.linearize(dev(m), dev(u), dev(adj))
    k, s = 8, 12
    bad = synth.omega(prob.n, s, seed=3)
    bad[5] = 0.0
    good = synth.omega(prob.n, s, seed=4)
    Vs = [dev(np.zeros((k, prob.n))) for _ in range(2)]
    lam_bad, info = gps[0].lowrank_eig(dev(bad), k, Vs[0])
    assert info["rc"] == 0, info
    lam_ref, _ = gps[1].lowrank_eig(dev(np.delete(bad, 5, axis=0)), k, Vs[1])
    e = np.max(np.abs(lam_bad - lam_ref)) / lam_ref[0]
    Vg = host(Vs[0]).T
    RV = np.column_stack([prob.R_apply(v) for v in Vg.T])
    print(f"[gpu-alg] zero probe column: |dlambda|/lambda_1 {e:.1e} against the 11-column block", flush=True)
    assert e <= 1e-8
    np.testing.assert_allclose(Vg.T @ RV, np.eye(k), atol=1e-8)
    worse = bad.copy()
    worse[:5] = 0.0     # rank 7 < k = 8
    with pytest.raises(hv.HinvError) as e:
        gps[0].lowrank_eig(dev(worse), k, Vs[0])
    assert e.value.code == hv.HINV_EBREAK
    b = hv.Batch(ctx, gps)
    with pytest.raises(hv.HinvError) as e:
        b.lowrank_eig([dev(good), dev(bad)], k, Vs)
    assert e.value.code == hv.HINV_EBREAK
    lam, info = b.lowrank_eig([dev(good), dev(good)], k, Vs)
    assert info["rc"] == 0
    np.testing.assert_allclose(lam[0], lam[1], rtol=0, atol=1e-12 * abs(lam[0][0]))


def test_double_pass_bf16_block_product(ctx, map32):
    prob, obs, m = map32
    k, p = 50, 20
    u = prob.forward(m)
    adj = prob.adjoint(m, u)
    Om = synth.omega(prob.n, k + p)
    A = lambda v: prob.hessian_apply(m, u, adj, v, model.HESS_MISFIT)
    lam_o, _, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om.T, k)
    gp = gpu_problem(ctx, prob, obs, hv.PREC_FP32_IR)
    gp.linearize(dev(m), dev(u), dev(adj))
    V = dev(np.zeros((k, prob.n)))
    lam, info = gp.lowrank_eig(dev(Om), k, V, tprod=hv.TPROD_BF16)
    err = np.abs(lam - lam_o) / abs(lam_o[0])
    print("[gpu] bf16 T: max |dlambda|/lambda_1 =", err.max(), "leading rel",
          abs(lam[0] - lam_o[0]) / lam_o[0], flush=True)
    # BF16 inputs (unit roundoff 2^-8) with FP32 accumulation: the projected
    # matrix is perturbed by ~ u_bf16 |T|, so eigenvalues move by ~ u_bf16 lambda_1.
    assert err.max() < 2e-2


def test_posterior_samples(ctx, map32):
    prob, obs, m = map32
    k, ns = 20, 6
    u = prob.forward(m)
    adj = prob.adjoint(m, u)
    Om = synth.omega(prob.n, k + 10)
    A = lambda v: prob.hessian_apply(m, u, adj, v, model.HESS_GN_MISFIT)
    lam, V, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om.T, k)
    eta = synth.white_noise(32, ns, stream=synth.STREAM_POST)
    ref = np.array([m + lowrank.posterior_sample_update(prob.KA_solve(prob.CM @ e), V, lam, prob.R_apply)
                    for e in eta])
    gp = gpu_problem(ctx, prob, obs)
    out = dev(np.zeros((ns, prob.n)))
    info = gp.posterior_sample(dev(m), lam, dev(V.T), dev(eta), out)
    assert info["rc"] == 0
    assert col_rel(host(out), ref) < 1e-8
    with pytest.raises(hv.HinvError) as e:
        gp.posterior_sample(dev(m), np.array([-1.5]), dev(V.T[:1]), dev(eta), out)
    assert e.value.code == hv.HINV_ENEGEIG


@pytest.mark.parametrize("N,first,ns", [(32, 0, 3), (256, 17, 2)])
def test_device_white_noise_matches_counter_definition(ctx, N, first, ns):
    prob, _, obs = instance(N, 10)
    gp = gpu_problem(ctx, prob, obs)
    eta = dev(np.zeros((ns, 6 * N * N)))
    gp.white_noise(1909, synth.STREAM_POST, first, eta)
    ref = synth.philox_white_noise(N, ns, seed=1909, stream=synth.STREAM_POST, first=first)
    assert np.max(np.abs(host(eta) - ref)) < 1e-13


def test_posterior_samples_from_device_noise(ctx, map32):
    prob, obs, m = map32
    k, ns = 12, 4
    u = prob.forward(m)
    adj = prob.adjoint(m, u)
    Om = synth.omega(prob.n, k + 8)
    A = lambda v: prob.hessian_apply(m, u, adj, v, model.HESS_GN_MISFIT)
    lam, V, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om.T, k)
    eta_o = synth.philox_white_noise(32, ns, seed=5, stream=synth.STREAM_POST, first=100)
    ref = np.array([m + lowrank.posterior_sample_update(prob.KA_solve(prob.CM @ e), V, lam, prob.R_apply)
                    for e in eta_o])
    gp = gpu_problem(ctx, prob, obs)
    eta = dev(np.zeros((ns, 6 * 32 * 32)))
    gp.white_noise(5, synth.STREAM_POST, 100, eta)
    out = dev(np.zeros((ns, prob.n)))
    gp.posterior_sample(dev(m), lam, dev(V.T), eta, out)
    assert col_rel(host(out), ref) < 1e-8


def test_seeded_posterior_samples_in_chunks(ctx, map32):
    """hinv_posterior_sample_seeded draws its noise on the device in chunks of
    256 samples: 300 samples (two chunks) equal the oracle's draws from the
    same counter-based noise, and a later range drawn alone equals the
    corresponding columns."""
    prob, obs, m = map32
    k, ns, first = 12, 300, 7
    u = prob.forward(m)
    adj = prob.adjoint(m, u)
    Om = synth.omega(prob.n, k + 8)
    A = lambda v: prob.hessian_apply(m, u, adj, v, model.HESS_GN_MISFIT)
    lam, V, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om.T, k)
    eta_o = synth.philox_white_noise(32, ns, seed=5, stream=synth.STREAM_POST, first=first)
    ref = np.array([m + lowrank.posterior_sample_update(prob.KA_solve(prob.CM @ e), V, lam, prob.R_apply)
                    for e in eta_o])
    gp = gpu_problem(ctx, prob, obs, hv.PREC_AUTO)
    out = dev(np.zeros((ns, prob.n)))
    info = gp.posterior_sample_seeded(dev(m), lam, dev(V.T), 5, synth.STREAM_POST, first, out)
    assert info["rc"] == 0, info
    got = host(out)
    print(f"[gpu] seeded samples: max column rel err {col_rel(got, ref):.2e}", flush=True)
    assert col_rel(got, ref) < 1e-8
    part = dev(np.zeros((4, prob.n)))
    gp.posterior_sample_seeded(dev(m), lam, dev(V.T), 5, synth.STREAM_POST, first + 260, part)
    assert col_rel(host(part), ref[260:264]) < 1e-8
