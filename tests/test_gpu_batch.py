"""GPU parity of batched independent inversions (uneven mesh sizes) against
the FP64 oracle, instance by instance.

Five instances with their own mesh size (4, 8, 16, 16, 32: one level, two
levels and deeper hierarchies, two instances sharing a size), prior
(gamma, delta), observation count and true field.  Bar as for single problems:
Hessian actions within 1e-8 (relative 2-norm per column) of the oracle in all
four modes; double-pass eigenvalues with the same probe matrix within
1e-8 lambda_1 of the oracle's.
"""
import numpy as np
import pytest

import synth
from cases import col_rel, instance
from oracle import lowrank, model

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hv = pytest.importorskip("paper_1909_03948_amd.hinv")

# (N, q, gamma, delta, seed)
SPECS = [(16, 40, 0.1, 0.5, 11), (4, 6, 0.2, 2.0, 12), (32, 100, 0.05, 1.0, 13),
         (8, 20, 0.15, 0.7, 14), (16, 60, 0.08, 1.5, 15)]


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def batch_setup():
    print("[gpu-batch] setup", flush=True)
    ctx = hv.Context(0)
    insts, gps = [], []
    for N, q, g, d, seed in SPECS:
        prob, _, obs = instance(N, q, g, d, seed)
        m = prob.m_pr + 0.5 * synth.smooth_field(N, seed=seed)
        u = prob.forward(m)
        p = prob.adjoint(m, u)
        gp = hv.Problem(ctx, N, g, d, obs_xy=obs, d_obs=prob.d, sigma=prob.sigma,
                        m_prior=prob.m_pr[0], beta=prob.beta, precision=hv.PREC_AUTO, rtol=1e-10)
        insts.append((prob, m, u, p))
        gps.append(gp)
    return ctx, insts, gps


def test_batch_requires_linearization(batch_setup):
    ctx, insts, gps = batch_setup
    b = hv.Batch(ctx, gps)
    mh = [dev(np.zeros((1, gp.n))) for gp in gps]
    with pytest.raises(hv.HinvError) as e:
        b.hessian_apply(hv.HESS_MISFIT, mh, mh)
    assert e.value.code == hv.HINV_ESTATE


@pytest.mark.parametrize("nrhs,shape", [(1, None), (3, None), (3, "l4c4"), (3, "s1c2")])
def test_batch_hessian_all_modes(batch_setup, nrhs, shape, monkeypatch):
    """Column blocks of 4 / 2 with 3 columns per problem straddle problems of a
    stacked hierarchy (their coefficient tiles are staged again)."""
    if shape:
        monkeypatch.setenv("HINV_SHAPE", shape)
    ctx, insts, gps = batch_setup
    for (prob, m, u, p), gp in zip(insts, gps):
        gp.linearize(dev(m), dev(u), dev(p))
    b = hv.Batch(ctx, gps)
    mh = [synth.test_vectors(prob.n, nrhs, stream=40 + i) for i, (prob, *_) in enumerate(insts)]
    outs = [dev(np.zeros((nrhs, prob.n))) for prob, *_ in insts]
    for mode in (hv.HESS_FULL, hv.HESS_MISFIT, hv.HESS_GN_FULL, hv.HESS_GN_MISFIT):
        print(f"[gpu-batch] hessian nrhs={nrhs} mode={mode}", flush=True)
        info = b.hessian_apply(mode, [dev(x) for x in mh], outs)
        assert info["rc"] == 0 and info["max_relres"] <= 1e-10, info
        for i, (prob, m, u, p) in enumerate(insts):
            ref = np.array([prob.hessian_apply(m, u, p, v, mode) for v in mh[i]])
            assert col_rel(host(outs[i]), ref) < 1e-8, (i, mode)


def test_batch_follows_relinearization(batch_setup):
    """A new linearization of one member is picked up by the batch."""
    ctx, insts, gps = batch_setup
    for (prob, m, u, p), gp in zip(insts, gps):
        gp.linearize(dev(m), dev(u), dev(p))
    b = hv.Batch(ctx, gps)
    mh = [dev(synth.test_vectors(prob.n, 2, stream=50 + i)) for i, (prob, *_) in enumerate(insts)]
    outs = [dev(np.zeros((2, prob.n))) for prob, *_ in insts]
    b.hessian_apply(hv.HESS_MISFIT, mh, outs)
    prob, m, u, p = insts[4]
    m2 = m + 0.3 * synth.smooth_field(prob.N, seed=99)
    u2 = prob.forward(m2)
    p2 = prob.adjoint(m2, u2)
    gps[4].linearize(dev(m2), dev(u2), dev(p2))
    b.hessian_apply(hv.HESS_MISFIT, mh, outs)
    ref = np.array([prob.hessian_apply(m2, u2, p2, v, model.HESS_MISFIT) for v in host(mh[4])])
    assert col_rel(host(outs[4]), ref) < 1e-8
    gps[4].linearize(dev(m), dev(u), dev(p))


@pytest.mark.parametrize("s", [14, 13])  # s <= n = 25 of the 4 x 4 mesh; odd s pads the Jacobi pairing
@pytest.mark.parametrize("mode", [hv.HESS_MISFIT, hv.HESS_GN_MISFIT])
def test_batch_double_pass(batch_setup, mode, s):
    ctx, insts, gps = batch_setup
    for (prob, m, u, p), gp in zip(insts, gps):
        gp.linearize(dev(m), dev(u), dev(p))
    b = hv.Batch(ctx, gps)
    k = 8
    oms = [synth.omega(prob.n, s, seed=200 + i) for i, (prob, *_) in enumerate(insts)]
    Vs = [dev(np.zeros((k, prob.n))) for prob, *_ in insts]
    lam, info = b.lowrank_eig([dev(o) for o in oms], k, Vs, mode=mode)
    assert info["rc"] == 0, info
    for i, (prob, m, u, p) in enumerate(insts):
        A = lambda v: prob.hessian_apply(m, u, p, v, mode)
        lam_o, _, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, oms[i].T, k)
        print(f"[gpu-batch] instance {i} N={prob.N}: lambda_1 {lam_o[0]:.3e} "
              f"max err {np.max(np.abs(lam[i] - lam_o)) / abs(lam_o[0]):.2e}", flush=True)
        assert np.max(np.abs(lam[i] - lam_o)) <= 1e-8 * abs(lam_o[0]), i
        Vg = host(Vs[i])
        G = Vg @ np.column_stack([prob.R_apply(v) for v in Vg])
        np.testing.assert_allclose(G, np.eye(k), atol=1e-8)


def test_batch_column_limit(batch_setup):
    ctx, insts, gps = batch_setup
    b = hv.Batch(ctx, gps)
    nrhs = 2049  # two problems share N = 16: 4098 columns > 4096
    mh = [dev(np.zeros((nrhs, prob.n))) for prob, *_ in insts]
    with pytest.raises(hv.HinvError) as e:
        b.hessian_apply(hv.HESS_MISFIT, mh, mh)
    assert e.value.code == hv.HINV_EINVAL


# meshes above the one-workgroup bottom (N > 32): the fused down/up V-cycle
# kernels run on stacked problems; two instances share N = 64
SPECS_LARGE = [(64, 120, 0.1, 0.8, 21), (128, 200, 0.06, 1.2, 22), (64, 80, 0.15, 0.6, 23)]


@pytest.fixture(scope="module")
def batch_large():
    print("[gpu-batch] large setup", flush=True)
    ctx = hv.Context(0)
    insts, gps = [], []
    for N, q, g, d, seed in SPECS_LARGE:
        prob, _, obs = instance(N, q, g, d, seed)
        m = prob.m_pr + 0.6 * synth.smooth_field(N, seed=seed)
        u = prob.forward(m)
        p = prob.adjoint(m, u)
        gp = hv.Problem(ctx, N, g, d, obs_xy=obs, d_obs=prob.d, sigma=prob.sigma,
                        m_prior=prob.m_pr[0], beta=prob.beta, precision=hv.PREC_AUTO, rtol=1e-10)
        gp.linearize(dev(m), dev(u), dev(p))
        insts.append((prob, m, u, p))
        gps.append(gp)
    return ctx, insts, gps


@pytest.mark.parametrize("shape", [None, "l4c4", "s1c3", "l16c8"])
def test_batch_hessian_stacked_large(batch_large, shape, monkeypatch):
    """Four columns per problem (FP32 refinement on the stacked N = 64 pair);
    column blocks of 3 and 8 straddle the two stacked problems.  Repeated calls
    check that the per-shape iteration estimate of the inner solves does not
    drift (every call converges to the requested tolerance)."""
    if shape:
        monkeypatch.setenv("HINV_SHAPE", shape)
    ctx, insts, gps = batch_large
    b = hv.Batch(ctx, gps)
    nrhs = 4
    mh = [synth.test_vectors(prob.n, nrhs, stream=70 + i) for i, (prob, *_) in enumerate(insts)]
    outs = [dev(np.zeros((nrhs, prob.n))) for prob, *_ in insts]
    for mode in (hv.HESS_MISFIT, hv.HESS_FULL):
        refs = [np.array([prob.hessian_apply(m, u, p, v, mode) for v in mh[i]])
                for i, (prob, m, u, p) in enumerate(insts)]
        for rep in range(3):
            print(f"[gpu-batch] large shape={shape} mode={mode} call {rep}", flush=True)
            info = b.hessian_apply(mode, [dev(x) for x in mh], outs)
            assert info["rc"] == 0 and info["max_relres"] <= 1e-10, info
            for i in range(len(insts)):
                assert col_rel(host(outs[i]), refs[i]) < 1e-8, (i, mode, rep)


# the uneven batch's largest sizes: two stacked N = 256 members and one at N = 512
SPECS_C5 = [(256, 300, 0.12, 0.9, 31), (512, 500, 0.07, 1.4, 32), (256, 150, 0.18, 1.8, 33)]


@pytest.fixture(scope="module")
def batch_c5():
    print("[gpu-batch] N = 256 / 512 setup", flush=True)
    ctx = hv.Context(0)
    insts, gps = [], []
    for N, q, g, d, seed in SPECS_C5:
        prob, _, obs = instance(N, q, g, d, seed)
        m = prob.m_pr + 0.6 * synth.smooth_field(N, seed=seed)
        u = prob.forward(m)
        p = prob.adjoint(m, u)
        gp = hv.Problem(ctx, N, g, d, obs_xy=obs, d_obs=prob.d, sigma=prob.sigma,
                        m_prior=prob.m_pr[0], beta=prob.beta, precision=hv.PREC_AUTO, rtol=1e-10)
        gp.linearize(dev(m), dev(u), dev(p))
        insts.append((prob, m, u, p))
        gps.append(gp)
    return ctx, insts, gps


def test_batch_hessian_and_double_pass_at_256_and_512(batch_c5):
    """The uneven batch's largest members: stacked N = 256 pair and N = 512,
    Hessian actions (FP32 refinement, 4 columns per member) within 1e-8 and
    double-pass eigenvalues within 1e-8 lambda_1 of the oracle."""
    ctx, insts, gps = batch_c5
    b = hv.Batch(ctx, gps)
    nrhs = 4
    mh = [synth.test_vectors(prob.n, nrhs, stream=80 + i) for i, (prob, *_) in enumerate(insts)]
    outs = [dev(np.zeros((nrhs, prob.n))) for prob, *_ in insts]
    info = b.hessian_apply(hv.HESS_GN_MISFIT, [dev(x) for x in mh], outs)
    assert info["rc"] == 0 and info["max_relres"] <= 1e-10, info
    for i, (prob, m, u, p) in enumerate(insts):
        ref = np.array([prob.hessian_apply(m, u, p, v, model.HESS_GN_MISFIT) for v in mh[i][:2]])
        e = col_rel(host(outs[i])[:2], ref)
        print(f"[gpu-batch] N={prob.N} Hessian action rel {e:.2e}", flush=True)
        assert e < 1e-8, i
    k, s = 8, 12
    oms = [synth.omega(prob.n, s, seed=300 + i) for i, (prob, *_) in enumerate(insts)]
    Vs = [dev(np.zeros((k, prob.n))) for prob, *_ in insts]
    lam, info = b.lowrank_eig([dev(o) for o in oms], k, Vs, mode=hv.HESS_GN_MISFIT)
    assert info["rc"] == 0, info
    for i, (prob, m, u, p) in enumerate(insts):
        A = lambda v: prob.hessian_apply(m, u, p, v, model.HESS_GN_MISFIT)
        lam_o, _, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, oms[i].T, k)
        err = np.max(np.abs(lam[i] - lam_o)) / abs(lam_o[0])
        print(f"[gpu-batch] N={prob.N}: lambda_1 {lam_o[0]:.3e} max err {err:.2e}", flush=True)
        assert err <= 1e-8, i
