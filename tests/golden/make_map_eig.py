"""Writes poisson{N}_map_oracle.npz: the oracle's MAP point and low-rank
eigenpairs for the N = 256 and N = 1024 workloads.

The GPU tests compare the library's Newton-CG MAP point (Alg. 1) and its
double-pass eigenpairs (Alg. 2 with PreCholQR, Alg. 4) against these values.
The oracle needs about a minute (N = 256) or a few hours (N = 1024) for them,
too long to repeat inside a GPU test, so this script evaluates them once.  It
calls only the oracle and the seeded input generators.

Instance: the workload's synthetic problem (true field a prior draw, data
B u(m_true) plus 1% noise, Sec. 5.1), built by ``oracle.model.make_instance``
from the ``synth`` draws of the master seed.

Stored:
  d_obs, sigma, beta            the data the GPU problem is given
  Newton record                 iterations, |g_i| history (oracle Newton-CG
                                from m_pr to |g| <= 1e-11 |g_0|)
  m_map - m_pr                  in full (N = 256) or, at N = 1024, its values
                                at 4 096 seeded indices, its 2-norm and its
                                inner products with two seeded Gaussian vectors
  lam_gn[k] (and lam_full[k] at N = 256)
                                eigenvalues of the Gauss-Newton (and full) data
                                misfit Hessian at m_map, B = R, probe matrix
                                synth.omega(n, k + p) with k + p columns
  v_gn_vals[10, 4096]           the leading ten eigenvectors (Gauss-Newton) at
                                the seeded indices, sign fixed so that the
                                sampled entry of largest magnitude is positive

Run: python tests/golden/make_map_eig.py 256     (about a minute)
     python tests/golden/make_map_eig.py 1024    (a few hours, ~25 GB)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import lowrank, model, newton  # noqa: E402

NSAMPLE = 4096
NLEAD = 10


def sign_fixed(V, idx):
    """Columns of V restricted to idx, each scaled by +-1 so that its entry of
    largest magnitude is positive."""
    S = V[idx, :]
    j = np.argmax(np.abs(S), axis=0)
    return (S * np.sign(S[j, np.arange(S.shape[1])])).T


def main(N: int):
    wl = {256: "poisson256", 1024: "poisson1024"}[N]
    cfg = synth.WORKLOADS[wl]
    path = os.path.join(HERE, f"poisson{N}_map_oracle.npz")
    t0 = time.time()
    log = lambda s: print(f"[{time.time() - t0:8.1f}s] {s}", flush=True)
    seed = synth.MASTER_SEED
    q = cfg["q"]
    prob, _, _ = model.make_instance(cfg, seed, synth.white_noise(N, seed=seed)[0],
                                     synth.obs_points(q, seed=seed), synth.obs_noise(q, seed=seed))
    n = prob.n
    log(f"instance N={N} n={n} q={q}")
    m_map, info = newton.newton_cg(prob, rel_tol=1e-11, verbose=True)
    log(f"newton: {info['iters']} iterations, converged={info['converged']} ({info['reason']}), "
        f"|g|/|g0| = {info['gnorm'][-1] / info['gnorm'][0]:.2e}")
    out = dict(N=N, q=q, gamma=cfg["gamma"], delta=cfg["delta"], beta=prob.beta, sigma=prob.sigma,
               d_obs=prob.d, newton_iters=info["iters"], newton_gnorm=np.array(info["gnorm"]),
               newton_converged=info["converged"], k=cfg["k"], p=cfg["p"])
    dm = m_map - prob.m_pr
    idx = synth.sample_indices(n, NSAMPLE)
    out["idx"] = idx
    if N <= 256:
        out["dm_full"] = dm
    else:
        W = synth.test_vectors(n, 2, stream=synth.STREAM_SAMPLE)
        out.update(dm_vals=dm[idx], dm_norm=np.linalg.norm(dm), dm_proj=W @ dm)
    out["dm_Rnorm"] = float(np.sqrt(dm @ prob.R_apply(dm)))
    u = prob.forward(m_map)
    p = prob.adjoint(m_map, u)
    k, s = cfg["k"], cfg["k"] + cfg["p"]
    Om = synth.omega(n, s).T
    modes = [("gn", model.HESS_GN_MISFIT)] + ([("full", model.HESS_MISFIT)] if N <= 256 else [])
    for name, mode in modes:
        A = lambda v: prob.hessian_apply(m_map, u, p, v, mode)
        lam, V, _ = lowrank.double_pass(A, prob.R_apply, prob.R_solve, Om, k)
        out[f"lam_{name}"] = lam
        if name == "gn":
            out["v_gn_vals"] = sign_fixed(V[:, :NLEAD], idx)
        log(f"double pass ({name}): lambda_1 {lam[0]:.6e} lambda_k {lam[-1]:.6e}")
    np.savez_compressed(path, **out)
    log(f"wrote {path}")


if __name__ == "__main__":
    main(int(sys.argv[1]))
