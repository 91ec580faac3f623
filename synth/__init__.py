"""Seeded synthetic inputs for the coefficient-inversion workloads.

This module draws the random numbers a run consumes and nothing else: white
noise for prior draws, observation locations, observation noise and the
Gaussian probe matrix of the randomized eigensolver.  It holds none of the
method's arithmetic, so both the CPU oracle and the GPU library can take its
output as input.

Every draw comes from NumPy's Philox4x64-10 bit generator keyed by
(seed, stream); the stream numbers below fix which draw is which, so two
callers with the same seed see bit-identical arrays.

Workload shapes follow the paper's Poisson example (Sec. 5.1): a unit-square
mesh, pointwise observations at uniformly drawn locations with i.i.d. Gaussian
noise, and a bilaplacian Gaussian prior.  The sizes are those of the workloads
listed in ``WORKLOADS``.
"""
from __future__ import annotations

import numpy as np

MASTER_SEED = 1909

# Stream identifiers (second Philox key word).
STREAM_TRUTH = 0      # white noise of the prior draw that serves as the true field
STREAM_OBS_POINTS = 1  # observation locations
STREAM_OBS_NOISE = 2  # observation noise
STREAM_OMEGA = 3      # Gaussian probe matrix of the randomized eigensolver
STREAM_POST = 4       # white noise of posterior samples
STREAM_TEST = 7       # generic test vectors (directions, right-hand sides)
STREAM_SAMPLE = 8     # sampled output indices and random functionals of large tests
STREAM_BATCH = 9      # sizes and prior parameters of the uneven batch

# Synthetic workloads shaped like the paper's Poisson example, scaled up.
WORKLOADS = {
    "poisson32": dict(N=32, q=100, gamma=0.1, delta=0.5, m_prior=-2.0, k=50, p=20),
    "poisson256": dict(N=256, q=400, gamma=0.1, delta=0.5, m_prior=-2.0, k=50, p=20),
    "poisson1024": dict(N=1024, q=2000, gamma=0.05, delta=1.0, m_prior=-2.0, k=200, p=20),
    # the paper's own Poisson setup (Sec. 5.1) on a P1 state: 64 x 64 cells
    # (4 225 parameters), 50 observations in [0.1, 0.9] x [0.1, 0.5],
    # anisotropic prior theta = (2, 0.5), alpha = pi/4
    # (rank r = 30 and oversampling l = 20 as in the section's low-rank posterior)
    "poisson64_paper": dict(N=64, q=50, gamma=0.1, delta=0.5, m_prior=-2.0, k=30, p=20,
                            theta=(2.0, 0.5, float(np.pi / 4)), obs_box=(0.1, 0.9, 0.1, 0.5),
                            state_degree=2),
}


def uneven_batch(count: int = 64, seed: int = MASTER_SEED, sizes=(64, 128, 256, 512),
                 q_range=(100, 1000), gamma_range=(0.05, 0.2), delta_range=(0.5, 2.0)) -> list:
    """Instances of the uneven batch: mesh size uniform over ``sizes``, gamma and
    delta uniform over their ranges, q uniform over the integers in q_range;
    instance i draws its own true field and data with seed + i."""
    g = _gen(seed, STREAM_BATCH)
    Ns = g.choice(np.asarray(sizes), size=count)
    gam = g.uniform(*gamma_range, size=count)
    dl = g.uniform(*delta_range, size=count)
    qs = g.integers(q_range[0], q_range[1] + 1, size=count)
    return [dict(N=int(Ns[i]), q=int(qs[i]), gamma=float(gam[i]), delta=float(dl[i]), m_prior=-2.0,
                 seed=seed + i) for i in range(count)]


def _gen(seed: int, stream: int) -> np.random.Generator:
    key = (int(seed) & ((1 << 64) - 1)) | ((int(stream) & ((1 << 64) - 1)) << 64)
    return np.random.Generator(np.random.Philox(key=key))


def n_nodes(N: int) -> int:
    return (N + 1) * (N + 1)


def n_noise(N: int) -> int:
    """Length of one white-noise vector: 3 edge-midpoint values per triangle."""
    return 6 * N * N


def white_noise(N: int, ns: int = 1, seed: int = MASTER_SEED,
                stream: int = STREAM_TRUTH) -> np.ndarray:
    """i.i.d. N(0,1) array of shape (ns, 6 N^2), one row per draw."""
    return _gen(seed, stream).standard_normal((ns, n_noise(N)))


def philox_white_noise(N: int, ns: int, seed: int = MASTER_SEED, stream: int = STREAM_POST,
                       first: int = 0) -> np.ndarray:
    """(ns, 6 N^2) standard normals from Philox4x64-10 with Box-Muller.

    Counter-based, so any sample can be drawn without the ones before it:
    sample s uses the words [s L, (s+1) L) of the Philox4x64-10 stream keyed by
    (seed, stream), L = 6 N^2; word w comes from counter block w // 4 + 1 (the
    stream NumPy's ``Philox`` produces).  Each word pair (w0, w1) gives
    u1 = ((w0 >> 11) + 1) 2^-53 in (0, 1], u2 = (w1 >> 11) 2^-53 in [0, 1) and
    the normals sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) (Box-Muller).
    The device generator of the library follows the same definition.
    """
    L = n_noise(N)
    if L % 4:
        raise ValueError("6 N^2 must be a multiple of 4 (N even)")
    out = np.empty((ns, L))
    key = (int(seed) & ((1 << 64) - 1)) | ((int(stream) & ((1 << 64) - 1)) << 64)
    for s in range(ns):
        g = np.random.Philox(key=key, counter=[(first + s) * (L // 4), 0, 0, 0])
        w = g.random_raw(L)
        u1 = ((w[0::2] >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
        u2 = (w[1::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        r = np.sqrt(-2.0 * np.log(u1))
        out[s, 0::2] = r * np.cos(2.0 * np.pi * u2)
        out[s, 1::2] = r * np.sin(2.0 * np.pi * u2)
    return out


def obs_points(q: int, seed: int = MASTER_SEED, lo: float = 0.05,
               hi: float = 0.95, box=None) -> np.ndarray:
    """(q, 2) locations drawn uniformly in [lo, hi]^2, or in the rectangle
    box = (x0, x1, y0, y1) when given."""
    if box is None:
        return _gen(seed, STREAM_OBS_POINTS).uniform(lo, hi, size=(q, 2))
    u = _gen(seed, STREAM_OBS_POINTS).uniform(0.0, 1.0, size=(q, 2))
    x0, x1, y0, y1 = box
    return np.column_stack([x0 + (x1 - x0) * u[:, 0], y0 + (y1 - y0) * u[:, 1]])


def obs_noise(q: int, seed: int = MASTER_SEED) -> np.ndarray:
    """(q,) i.i.d. N(0,1) draws that scale into observation noise."""
    return _gen(seed, STREAM_OBS_NOISE).standard_normal(q)


def omega(n: int, b: int, seed: int = MASTER_SEED) -> np.ndarray:
    """Gaussian probe matrix stored column by column: shape (b, n)."""
    return _gen(seed, STREAM_OMEGA).standard_normal((b, n))


def test_vectors(n: int, b: int, seed: int = MASTER_SEED,
                 stream: int = STREAM_TEST, scale: float = 1.0) -> np.ndarray:
    """(b, n) i.i.d. N(0, scale^2) vectors for directions and right-hand sides."""
    return scale * _gen(seed, stream).standard_normal((b, n))


def sample_indices(n: int, count: int, seed: int = MASTER_SEED) -> np.ndarray:
    """Sorted distinct indices in [0, n), drawn uniformly (sampled outputs of large tests)."""
    return np.sort(_gen(seed, STREAM_SAMPLE).choice(n, size=min(count, n), replace=False))


def smooth_field(N: int, seed: int = MASTER_SEED, stream: int = STREAM_TEST,
                 modes: int = 4, amp: float = 0.5) -> np.ndarray:
    """Nodal values of a random smooth trigonometric field (for tests only).

    f(x, y) = sum_{a,b < modes} c_ab cos(pi a x) cos(pi b y) / (1 + a^2 + b^2)
    with c_ab ~ N(0, amp^2).  Returned in node order k = j (N+1) + i.
    """
    g = _gen(seed, stream)
    c = amp * g.standard_normal((modes, modes))
    x = np.linspace(0.0, 1.0, N + 1)
    X, Y = np.meshgrid(x, x)  # Y varies along rows: X[j, i] = x_i, Y[j, i] = y_j
    f = np.zeros_like(X)
    for a in range(modes):
        for b in range(modes):
            f += c[a, b] * np.cos(np.pi * a * X) * np.cos(np.pi * b * Y) / (1.0 + a * a + b * b)
    return f.reshape(-1)
