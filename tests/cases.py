"""Shared construction of seeded test instances (oracle side + GPU-side inputs).

The oracle builds the synthetic instance (true field as a prior draw, data
from its forward solve plus seeded noise); the GPU problem receives the same
observation points, data and noise level.  No input or expected value comes
from the HIP path.
"""
from __future__ import annotations

import functools

import numpy as np

import synth
from oracle import model


@functools.lru_cache(maxsize=8)
def instance(N: int, q: int, gamma: float = 0.1, delta: float = 0.5, seed: int = synth.MASTER_SEED,
             state_degree: int = 1):
    cfg = dict(N=N, q=q, gamma=gamma, delta=delta, m_prior=-2.0, state_degree=state_degree)
    prob, m_true, u_true = model.make_instance(
        cfg, seed, synth.white_noise(N, seed=seed)[0], synth.obs_points(q, seed=seed),
        synth.obs_noise(q, seed=seed))
    return prob, m_true, synth.obs_points(q, seed=seed)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def col_rel(A, B):
    """Largest per-column relative 2-norm difference of (c, n) arrays."""
    return max(rel(a, b) for a, b in zip(np.atleast_2d(A), np.atleast_2d(B)))


def col_maxabs(A, B):
    """Largest per-column max-entry difference relative to the column's largest
    entry of B: an error confined to a few rows (a boundary row, a tile edge)
    shows here at full size while the 2-norm dilutes it."""
    A, B = np.atleast_2d(A), np.atleast_2d(B)
    out = 0.0
    for a, b in zip(A, B):
        den = np.max(np.abs(b))
        out = max(out, np.max(np.abs(a - b)) / (den if den > 0 else 1.0))
    return out
