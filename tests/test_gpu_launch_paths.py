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


@pytest.mark.parametrize("max_iter", [2, 3, 5, 6])
def test_iteration_cap_same_iterate_on_graph_and_eager_paths(ctx, max_iter, monkeypatch):
    """With the iteration cap inside the run that the prologue graph carries,
    the graph path (prologue plus a run shortened to the cap) and the eager
    path stop at the same iterate: the state solve reports HINV_ENOCONV with
    identical outputs, and a solve after lifting the cap reaches 1e-10 on
    both paths."""
    print(f"[gpu-paths] max_iter={max_iter}", flush=True)
    prob, gp = linearized(ctx, 64, 120)
    b = synth.test_vectors(prob.n, 1, stream=81)
    b[:, ~prob.free] = 0.0
    bd = dev(b)
    # a solve without the cap first: its iteration count sets the length of
    # the run before the first completion check
    x0 = torch.zeros_like(bd)
    assert gp.state_solve(bd, x0)["rc"] == 0
    outs = []
    for eager in (False, True):
        if eager:
            monkeypatch.setenv("HINV_NO_GRAPHS", "1")
        gp.set_solver(hv.PREC_FP64, 1e-10, max_iter)
        x = torch.zeros_like(bd)
        info = gp.state_solve(bd, x)
        torch.cuda.synchronize()
        assert info["rc"] == hv.HINV_ENOCONV, info
        outs.append((x.cpu().numpy(), info["iterations"]))
        gp.set_solver(hv.PREC_FP64, 1e-10, 0)
        x = torch.zeros_like(bd)
        info = gp.state_solve(bd, x)
        assert info["rc"] == 0 and info["max_relres"] <= 1e-10, info
        monkeypatch.delenv("HINV_NO_GRAPHS", raising=False)
    assert outs[0][1] == outs[1][1], outs
    assert np.array_equal(outs[0][0], outs[1][0])
