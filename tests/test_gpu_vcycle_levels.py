"""Several coarse levels a launch change no result.

With few columns the coarse levels of a V-cycle are latency bound, so the
down steps of two coarse levels share one launch and the up steps of up to
four another, each workgroup recomputing the coarser values its tile needs on
a larger tile.  The arithmetic per node is that of the one-level kernels, in
the same order, so Hessian actions and prior solves agree bit for bit with
one level a launch (HINV_NO_PAIRS, read when a problem is built) and take the
same iterations.  The mesh sizes cover no multi-level launch (N = 128), one
down pair with a two-level up chain (256), a down pair under a three-level
chain (512), a four-level chain with the wide finest tiles (1024) and a
four-level chain with one more level above it (2048); three columns cover the
small-tile path with several columns, the FP32-refined precision the
single-precision cycle vectors of its PCG.  The two largest meshes are
linearized on the device alone (the comparison needs no oracle).
"""
import numpy as np
import pytest

import synth
from cases import instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hv = pytest.importorskip("paper_1909_03948_amd.hinv")


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def ctx():
    return hv.Context(0)


def build(ctx, N, q, precision, one_level, monkeypatch):
    prob, _, obs = instance(N, q)
    m = prob.m_pr + 0.6 * synth.smooth_field(N, seed=5)
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    if one_level:
        monkeypatch.setenv("HINV_NO_PAIRS", "1")
    else:
        monkeypatch.delenv("HINV_NO_PAIRS", raising=False)
    gp = hv.Problem(ctx, N, prob.gamma, prob.delta, obs_xy=obs, d_obs=prob.d, sigma=prob.sigma,
                    m_prior=prob.m_pr[0], beta=prob.beta, precision=precision, rtol=1e-10)
    monkeypatch.delenv("HINV_NO_PAIRS", raising=False)
    gp.linearize(dev(m), dev(u), dev(p))
    return prob, gp


def actions(gp, x):
    h = torch.zeros_like(x)
    z = torch.zeros_like(x)
    ih = gp.hessian_apply(hv.HESS_FULL, x, h)
    iz = gp.prior_solve(x, z)
    assert ih["rc"] == 0 and iz["rc"] == 0, (ih, iz)
    torch.cuda.synchronize()
    return h.cpu().numpy(), z.cpu().numpy(), ih["iterations"], iz["iterations"]


@pytest.mark.parametrize("N,q,nc,prec", [(128, 200, 1, "fp64"), (256, 400, 1, "fp64"), (512, 600, 1, "fp64"),
                                         (256, 400, 3, "fp64"), (512, 600, 2, "fp32ir")])
def test_multi_level_launches_match_one_level_launches(ctx, N, q, nc, prec, monkeypatch):
    print(f"[gpu-vcycle-levels] N={N} nc={nc} {prec}", flush=True)
    precision = {"fp64": hv.PREC_FP64, "fp32ir": hv.PREC_FP32_IR}[prec]
    prob, multi = build(ctx, N, q, precision, False, monkeypatch)
    _, single = build(ctx, N, q, precision, True, monkeypatch)
    x = dev(synth.test_vectors(prob.n, nc, stream=81))
    h1, z1, ih1, iz1 = actions(single, x)
    h2, z2, ih2, iz2 = actions(multi, x)
    print(f"  iterations {ih1}/{iz1} vs {ih2}/{iz2}; max diff {np.max(np.abs(h2 - h1)):.1e} {np.max(np.abs(z2 - z1)):.1e}",
          flush=True)
    assert (ih1, iz1) == (ih2, iz2)
    assert np.array_equal(h1, h2)
    assert np.array_equal(z1, z2)


def build_device_only(ctx, N, q, one_level, monkeypatch):
    if one_level:
        monkeypatch.setenv("HINV_NO_PAIRS", "1")
    else:
        monkeypatch.delenv("HINV_NO_PAIRS", raising=False)
    gp = hv.Problem(ctx, N, 0.05, 1.0, obs_xy=synth.obs_points(q), d_obs=synth.obs_noise(q), sigma=0.01,
                    m_prior=-2.0, precision=hv.PREC_FP64, rtol=1e-10)
    monkeypatch.delenv("HINV_NO_PAIRS", raising=False)
    n = (N + 1) ** 2
    m = dev(-2.0 + 0.6 * synth.smooth_field(N, seed=5))
    u, p, g = (torch.zeros(n, dtype=torch.float64, device="cuda") for _ in range(3))
    gp.forward(m, u)
    gp.gradient(m, u, p, g)
    gp.linearize(m, u, p)
    return gp, n


@pytest.mark.parametrize("N,nc", [(1024, 1), (1024, 3), (2048, 1)])
def test_multi_level_launches_match_at_large_meshes(ctx, N, nc, monkeypatch):
    print(f"[gpu-vcycle-levels] device-only N={N} nc={nc}", flush=True)
    multi, n = build_device_only(ctx, N, 400, False, monkeypatch)
    single, _ = build_device_only(ctx, N, 400, True, monkeypatch)
    x = dev(synth.test_vectors(n, nc, stream=82))
    h1, z1, ih1, iz1 = actions(single, x)
    h2, z2, ih2, iz2 = actions(multi, x)
    print(f"  iterations {ih1}/{iz1} vs {ih2}/{iz2}; max diff {np.max(np.abs(h2 - h1)):.1e} {np.max(np.abs(z2 - z1)):.1e}",
          flush=True)
    assert (ih1, iz1) == (ih2, iz2)
    assert np.array_equal(h1, h2)
    assert np.array_equal(z1, z2)
