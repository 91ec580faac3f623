"""Pins of the CNN / flexible-CG oracle (no GPU).

* conv equals SciPy's 2-D cross-correlation summed over input channels;
* the backward pass matches central finite differences of the loss;
* the first Adam step is -lr g / (|g| + eps) elementwise (bias correction);
* the bf16 rounding equals torch's float32 -> bfloat16 conversion;
* flexible CG with a fixed SPD preconditioner reproduces preconditioned CG
  iterate by iterate, and with the identity solves an n x n system in <= n steps.
"""
import numpy as np
import pytest
from scipy import signal

from oracle import cnn

SMALL = [(4, 3), (4, 4), (4, 4), (4, 4), (4, 4), (1, 4)]


def rng(s=0):
    return np.random.default_rng(s)


def test_conv_is_cross_correlation():
    g = rng(1)
    x = g.standard_normal((2, 3, 7, 5))
    W = g.standard_normal((4, 3, 3, 3))
    b = g.standard_normal(4)
    y = cnn.conv(x, W, b)
    for bi in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate2d(x[bi, c], W[o, c], mode="same") for c in range(3))
            np.testing.assert_allclose(y[bi, o], ref, rtol=1e-12, atol=1e-12)


def test_gradient_matches_finite_differences():
    g = rng(2)
    theta = cnn.init_params(g, SMALL, scale=1.5)
    theta += 0.05 * g.standard_normal(theta.size)  # nonzero biases
    x = g.standard_normal((2, 3, 6, 5))
    t = g.standard_normal((2, 1, 6, 5))
    L, grad = cnn.gradient(theta, x, t, shapes=SMALL)
    eps = 1e-6
    for idx in g.choice(theta.size, size=25, replace=False):
        e = np.zeros_like(theta)
        e[idx] = eps
        Lp, _ = cnn.loss(cnn.forward(theta + e, x, shapes=SMALL)[0], t)
        Lm, _ = cnn.loss(cnn.forward(theta - e, x, shapes=SMALL)[0], t)
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, grad[idx])


def test_energy_gradient_matches_finite_differences():
    g = rng(12)
    theta = cnn.init_params(g, SMALL, scale=1.5)
    theta += 0.05 * g.standard_normal(theta.size)
    x = g.standard_normal((2, 3, 6, 5))
    x[:, 2] = (g.random((2, 6, 5)) > 0.2).astype(float)  # free-node mask
    t = np.concatenate([g.standard_normal((2, 1, 6, 5)), 0.5 + g.random((2, 2, 6, 5)),
                        np.zeros((2, 1, 6, 5))], axis=1)
    t[:, 3] = 2.5 + g.random((2, 6, 5))  # diagonally dominant: positive definite
    L, grad = cnn.gradient(theta, x, t, shapes=SMALL)
    eps = 1e-6
    for idx in g.choice(theta.size, size=25, replace=False):
        e = np.zeros_like(theta)
        e[idx] = eps
        Lp, _ = cnn.energy_loss(cnn.forward(theta + e, x, shapes=SMALL)[0], t, x[:, 2:3])
        Lm, _ = cnn.energy_loss(cnn.forward(theta - e, x, shapes=SMALL)[0], t, x[:, 2:3])
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - grad[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, grad[idx])


def test_stencil_is_the_assembled_matrix():
    """stencil_apply equals the sparse 5-point matrix built edge by edge."""
    g = rng(13)
    H, W = 5, 4
    wE, wN = g.random((H, W)), g.random((H, W))
    dg = 3.0 + g.random((H, W))
    A = np.diag(dg.reshape(-1))
    idx = lambda r, c: r * W + c
    for r in range(H):
        for c in range(W):
            if c + 1 < W:
                A[idx(r, c), idx(r, c + 1)] = A[idx(r, c + 1), idx(r, c)] = -wE[r, c]
            if r + 1 < H:
                A[idx(r, c), idx(r + 1, c)] = A[idx(r + 1, c), idx(r, c)] = -wN[r, c]
    v = g.standard_normal((H, W))
    np.testing.assert_allclose(cnn.stencil_apply(v, wE, wN, dg).reshape(-1), A @ v.reshape(-1), rtol=1e-13)


def test_first_adam_step():
    g = rng(3)
    th = g.standard_normal(50)
    gr = g.standard_normal(50)
    new, m, v = cnn.adam_step(th, gr, np.zeros(50), np.zeros(50), 1, lr=1e-2)
    np.testing.assert_allclose(new, th - 1e-2 * gr / (np.abs(gr) + cnn.ADAM_EPS), rtol=1e-12)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    g = rng(4)
    x = np.concatenate([g.standard_normal(1000) * 10.0 ** g.integers(-5, 5, 1000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(x), ref)


def test_fcg_with_fixed_preconditioner_is_pcg():
    g = rng(5)
    n = 30
    Q = g.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    Pm = np.diag(1.0 / np.diag(A))
    b = g.standard_normal(n)
    # textbook PCG, iterate by iterate
    x = np.zeros(n)
    r = b.copy()
    z = Pm @ r
    p = z.copy()
    xs = []
    for _ in range(8):
        q = A @ p
        a = (r @ z) / (p @ q)
        x = x + a * p
        rn = r - a * q
        zn = Pm @ rn
        p = zn + (rn @ zn) / (r @ z) * p
        r, z = rn, zn
        xs.append(x.copy())
    for k in range(1, 9):
        xf, it, _ = cnn.fcg(lambda v: A @ v, b, lambda v: Pm @ v, rtol=0.0, max_iter=k)
        assert it == k
        np.testing.assert_allclose(xf, xs[k - 1], rtol=1e-10, atol=1e-12)


def test_fcg_identity_solves_in_n_steps():
    g = rng(6)
    n = 12
    Q = g.standard_normal((n, n))
    A = Q @ Q.T + np.eye(n)
    b = g.standard_normal(n)
    x, it, hist = cnn.fcg(lambda v: A @ v, b, lambda v: v, rtol=1e-10, max_iter=3 * n)
    assert it <= n + 2
    np.testing.assert_allclose(A @ x, b, atol=1e-8)
