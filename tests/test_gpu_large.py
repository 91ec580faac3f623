"""GPU parity at the full size of the 1024 x 1024 workload (1 050 625
parameters, 2 000 observations, gamma = 0.05, delta = 1), in the launch
configuration its benchmark uses (batched FP32 solves inside FP64 refinement,
220 probe vectors, k = 200).

The oracle needs minutes per sparse factorisation at this size, so its values
come from ``golden/poisson1024_oracle.npz``, written by
``golden/make_poisson1024.py`` (oracle and seeded generators only): the data
vector, and per output the values at 4 096 seeded indices, the 2-norm and the
inner products with two standard-normal vectors w.  Bar, each relative to the
output's norm: sampled entries, the norm, and |<w, gpu - oracle>| (an unbiased
estimate of the 2-norm error in which every entry takes part) within 1e-8;
the Hessian action at the benchmark's 1e-10 residual included, in both of
its launch forms (8 columns in FP32 refinement, one column in FP64 PCG).  The eigensolver is checked
by properties that hold at any size, through operators whose parity the first
test establishes: R-orthonormality of V, Ritz values equal to the Rayleigh
quotients v^T H v of their vectors, and eigen-residuals
|H v - lambda R v|_{R^-1} / lambda of the leading pairs below sqrt(lambda_k / lambda) (the norm of the
generalized problem; the Euclidean norm would weigh the high frequencies by the
h^-4 spread of R's spectrum).
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
hv = pytest.importorskip("paper_1909_03948_amd.hinv")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "poisson1024_oracle.npz")


@pytest.fixture(scope="module")
def big():
    print("[gpu-large] N=1024 problem", flush=True)
    z = dict(np.load(GOLDEN))
    N = int(z["N"])
    ctx = hv.Context(0)
    gp = hv.Problem(ctx, N, float(z["gamma"]), float(z["delta"]), obs_xy=synth.obs_points(int(z["q"])),
                    d_obs=z["d_obs"], sigma=float(z["sigma"]), m_prior=-2.0, beta=float(z["beta"]),
                    precision=hv.PREC_AUTO, rtol=1e-10)
    n = (N + 1) ** 2
    m = -2.0 + 0.6 * synth.smooth_field(N, seed=4)
    W = synth.test_vectors(n, 2, stream=synth.STREAM_SAMPLE)
    return z, gp, m, W, ctx


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def check(z, W, name, v, tol=1e-8):
    idx = z["idx"]
    nrm = float(z[f"{name}_norm"])
    err_s = np.max(np.abs(v[idx] - z[f"{name}_vals"])) / nrm
    err_n = abs(np.linalg.norm(v) - nrm) / nrm
    # w ~ N(0, I): <w, e> ~ N(0, |e|^2), so |<w, v - ref>| / |ref| estimates the
    # relative 2-norm error with every entry taking part
    err_p = np.max(np.abs(W @ v - z[f"{name}_proj"])) / nrm
    print(f"[gpu-large] {name}: sampled {err_s:.2e} norm {err_n:.2e} functionals {err_p:.2e}", flush=True)
    assert err_s < tol and err_n < tol and err_p < tol, name


def test_forward_gradient_hessian_at_full_size(big):
    z, gp, m, W, _ = big
    n = m.size
    md, ud, pd, gd = dev(m), dev(np.zeros(n)), dev(np.zeros(n)), dev(np.zeros(n))
    info = gp.forward(md, ud)
    assert info["rc"] == 0 and info["max_relres"] <= 1e-10, info
    check(z, W, "u", host(ud))
    mis, reg = gp.cost(md, ud)
    assert abs(mis - z["misfit"]) <= 1e-8 * abs(z["misfit"])
    assert abs(reg - z["reg"]) <= 1e-10 * abs(z["reg"])
    gp.gradient(md, ud, pd, gd)
    check(z, W, "p", host(pd))
    check(z, W, "g", host(gd))
    gp.linearize(md, ud, pd)
    mh = synth.test_vectors(n, 8, stream=31)
    # A Hessian action chains two solves (the right-hand side of p-hat holds
    # u-hat).  With both FP32-refined solves stopped at 1e-10 its error was
    # 1.3e-8 here; the library runs the first of them to 1e-11 in that form,
    # and the bar is 1e-8 at the benchmark's 1e-10.
    for nc, cols in ((8, (0, 5)), (1, (0,))):   # FP32 refinement / FP64 PCG
        print(f"[gpu-large] Hessian action, {nc} column(s)", flush=True)
        out = dev(np.zeros((nc, n)))
        info = gp.hessian_apply(hv.HESS_MISFIT, dev(mh[:nc]), out)
        assert info["rc"] == 0 and info["max_relres"] <= 1e-10, info
        got = host(out)
        for c in cols:
            check(z, W, f"h{c}", got[c])


def test_eigenpairs_at_full_size_by_properties(big):
    z, gp, m, W, _ = big
    n = m.size
    u, p, g = dev(np.zeros(n)), dev(np.zeros(n)), dev(np.zeros(n))
    md = dev(m)
    gp.forward(md, u)
    gp.gradient(md, u, p, g)
    gp.linearize(md, u, p)
    k, s = 200, 220
    V = dev(np.zeros((k, n)))
    lam, info = gp.lowrank_eig(dev(synth.omega(n, s)), k, V, mode=hv.HESS_GN_MISFIT)
    assert info["rc"] == 0, info
    print(f"[gpu-large] lambda_1 {lam[0]:.4e} lambda_k {lam[-1]:.4e}", flush=True)
    assert np.all(np.diff(lam) <= 0) and lam[0] > 0
    RV = dev(np.zeros((k, n)))
    gp.prior_apply(V, RV)
    G = (V @ RV.T).cpu().numpy()
    print(f"[gpu-large] |V^T R V - I|_max {np.max(np.abs(G - np.eye(k))):.2e}", flush=True)
    np.testing.assert_allclose(G, np.eye(k), atol=1e-8)
    lead = 8
    lt = torch.as_tensor(lam[:lead], device="cuda")
    HV = dev(np.zeros((lead, n)))
    gp.hessian_apply(hv.HESS_GN_MISFIT, V[:lead].contiguous(), HV)
    # Ritz values are the Rayleigh quotients of the Ritz vectors (v^T R v = 1)
    rq = ((HV * V[:lead]).sum(dim=1) / lt - 1.0).abs().cpu().numpy()
    print("[gpu-large] leading |v^T H v / lambda - 1|", np.array2string(rq, precision=2), flush=True)
    assert np.all(rq < 1e-8), rq
    # residual in the norm of the generalized problem: |H v - lambda R v|_{R^-1} / lambda
    Rres = (HV - lt[:, None] * RV[:lead]).contiguous()
    Y = dev(np.zeros((lead, n)))
    gp.prior_solve(Rres, Y)
    res = ((Rres * Y).sum(dim=1).clamp(min=0).sqrt() / lt).cpu().numpy()
    print("[gpu-large] leading eigen-residuals (R^-1 norm)", np.array2string(res, precision=2), flush=True)
    # Rayleigh-Ritz on the sampled subspace Q: the residual of a Ritz pair is
    # (I - P_Q) H P_Q v, of size about sqrt(lambda_{s+1} lambda_j) once Q holds the
    # leading eigenspace, so residual_j / lambda_j <~ sqrt(lambda_{s+1} / lambda_j)
    # <= sqrt(lambda_k / lambda_j)
    bound = np.sqrt(lam[-1] / lam[:lead])
    assert np.all(res < bound), (res, bound)


def test_posterior_samples_at_full_size(big):
    z, gp, m, W, _ = big
    n = m.size
    N = int(z["N"])
    V = synth.test_vectors(n, 10, stream=32, scale=1e-3)
    lam = np.linspace(50.0, 0.5, 10)
    eta = dev(np.zeros((2, 6 * N * N)))
    gp.white_noise(77, synth.STREAM_POST, 3, eta)
    out = dev(np.zeros((2, n)))
    info = gp.posterior_sample(dev(m), lam, dev(V), eta, out)
    assert info["rc"] == 0, info
    got = host(out)
    for j in range(2):
        check(z, W, f"post{j}", got[j])
