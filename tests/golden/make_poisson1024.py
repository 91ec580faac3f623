"""Writes poisson1024_oracle.npz: oracle values for the 1024 x 1024 workload.

At this size the oracle needs minutes per sparse factorisation, too long to
repeat inside a GPU test, so this script evaluates it once and stores the data
vector and sampled outputs.  It calls only the oracle and the seeded input
generators.  Stored per quantity: the values at 4 096 seeded node indices, the
2-norm, and the inner products with two seeded Gaussian vectors (global
functionals that see every entry).

Quantities, at m = m_pr + 0.6 smooth_field(seed=4):
  u (forward), p (adjoint), g (gradient), misfit and regularization terms,
  H_misfit mh_c for probe columns c = 0, 5 of test_vectors(n, 8, stream=31),
  posterior samples m + (I - V S V^T R) K_A^{-1} C_M eta_j for V =
  test_vectors(n, 10, stream=32, scale=1e-3), lambda = linspace(50, 0.5, 10)
  and eta_j the counter-based white noise (seed 77, first sample 3), j = 0, 1.

Run: python tests/golden/make_poisson1024.py   (about 10 minutes, ~20 GB)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import lowrank, model  # noqa: E402

N, Q, GAMMA, DELTA = 1024, 2000, 0.05, 1.0
NSAMPLE = 4096


def summary(v, idx, W):
    return dict(vals=v[idx], norm=np.linalg.norm(v), proj=W @ v)


def main(path=os.path.join(HERE, "poisson1024_oracle.npz")):
    t0 = time.time()
    log = lambda s: print(f"[{time.time() - t0:7.1f}s] {s}", flush=True)
    cfg = dict(N=N, q=Q, gamma=GAMMA, delta=DELTA, m_prior=-2.0)
    seed = synth.MASTER_SEED
    prob, m_true, _ = model.make_instance(cfg, seed, synth.white_noise(N, seed=seed)[0],
                                          synth.obs_points(Q, seed=seed), synth.obs_noise(Q, seed=seed))
    log("instance")
    n = prob.n
    idx = synth.sample_indices(n, NSAMPLE)
    W = synth.test_vectors(n, 2, stream=synth.STREAM_SAMPLE)
    m = prob.m_pr + 0.6 * synth.smooth_field(N, seed=4)
    out = dict(N=N, q=Q, gamma=GAMMA, delta=DELTA, beta=prob.beta, sigma=prob.sigma,
               d_obs=prob.d, idx=idx)
    u = prob.forward(m)
    log("forward")
    p = prob.adjoint(m, u)
    g = prob.gradient(m, u, p)
    _, mis, reg = prob.cost(m, u)
    out.update(misfit=mis, reg=reg)
    for name, v in (("u", u), ("p", p), ("g", g)):
        for key, val in summary(v, idx, W).items():
            out[f"{name}_{key}"] = val
    mh = synth.test_vectors(n, 8, stream=31)
    for c in (0, 5):
        h = prob.hessian_apply(m, u, p, mh[c], model.HESS_MISFIT)
        for key, val in summary(h, idx, W).items():
            out[f"h{c}_{key}"] = val
    log("hessian")
    V = synth.test_vectors(n, 10, stream=32, scale=1e-3).T
    lam = np.linspace(50.0, 0.5, 10)
    eta = synth.philox_white_noise(N, 2, seed=77, stream=synth.STREAM_POST, first=3)
    for j in range(2):
        x = prob.KA_solve(prob.CM @ eta[j])
        s = m + lowrank.posterior_sample_update(x, V, lam, prob.R_apply)
        for key, val in summary(s, idx, W).items():
            out[f"post{j}_{key}"] = val
    log("posterior samples")
    np.savez_compressed(path, **out)
    log(f"wrote {path}")


if __name__ == "__main__":
    main()
