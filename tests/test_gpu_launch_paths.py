"""The solver's launch paths give identical results.

A solve runs its prologue and the PCG iterations as captured graphs; with
the kernel timer on, every 16th solve runs two iterations eagerly (each
launch carrying an event pair); with HINV_NO_GRAPHS every launch is eager.
The kernels and their order are the same on every path, and kernels of
finished columns return at once, so the outputs must agree bit for bit.
"""
import numpy as np
import pytest

import synth
from cases import instance

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hv = pytest.importorskip("paper_1909_03948_amd.hinv")

CLASSES = ["mg_down", "mg_up", "mg_bottom", "pcg_apply", "pcg_update"]


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def ctx():
    return hv.Context(0)


def linearized(ctx, N, q):
    prob, _, obs = instance(N, q)
    m = prob.m_pr + 0.6 * synth.smooth_field(N, seed=5)
    u = prob.forward(m)
    p = prob.adjoint(m, u)
    gp = hv.Problem(ctx, N, prob.gamma, prob.delta, obs_xy=obs, d_obs=prob.d, sigma=prob.sigma,
                    m_prior=prob.m_pr[0], beta=prob.beta, precision=hv.PREC_AUTO, rtol=1e-10)
    gp.linearize(dev(m), dev(u), dev(p))
    return prob, gp


def run(gp, mh, reps):
    outs = []
    for _ in range(reps):
        out = torch.zeros_like(mh)
        info = gp.hessian_apply(hv.HESS_FULL, mh, out)
        assert info["rc"] == 0, info
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
    return outs


@pytest.mark.parametrize("N,q,nc", [(64, 120, 1), (256, 400, 1), (64, 120, 9)])
def test_timed_and_eager_paths_match_graph_path(ctx, N, q, nc, monkeypatch):
    print(f"[gpu-paths] N={N} nc={nc}", flush=True)
    prob, gp = linearized(ctx, N, q)
    mh = dev(synth.test_vectors(prob.n, nc, stream=80))
    ref = run(gp, mh, 2)
    assert np.array_equal(ref[0], ref[1])
    # timer on: 12 Hessian actions = 24 solves, so some solves take the sampled path
    for c in CLASSES:
        ctx.kernel_timer(c, True, 16)
    timed = run(gp, mh, 12)
    sampled = sum(ctx.kernel_timer_read(c)["timed"] for c in CLASSES)
    for c in CLASSES:
        ctx.kernel_timer(c, False, 16)
    assert sampled > 0
    for o in timed:
        assert np.array_equal(o, ref[0])
    monkeypatch.setenv("HINV_NO_GRAPHS", "1")
    eager = run(gp, mh, 1)
    assert np.array_equal(eager[0], ref[0])
