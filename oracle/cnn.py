"""FP64 oracle of the learned preconditioner's network, its training step and
flexible CG (TEST INFRASTRUCTURE ONLY: used by tests and the benchmark's CPU
baseline, never by the library).

Network (a 6-layer residual CNN on the nodal grid, zero padding, 3x3 kernels,
32 channels):
    h0 = relu(conv(x, W0) + b0)                 3 -> 32 channels
    h_l = h_{l-1} + relu(conv(h_{l-1}, W_l) + b_l),   l = 1..4
    y  = conv(h4, W5) + b5                      32 -> 1 channel
conv is cross-correlation: conv(x, W)[o, i, j] = sum_{c, a, b} W[o, c, a, b]
x[c, i + a - 1, j + b - 1] with x = 0 outside the image.  Images are indexed
[row j][column i] = node (i, j) of the mesh.

Loss over a batch: mean over samples of |y - t|^2 / |t|^2 (relative L2), or of
(y - t)^T A (y - t) / t^T A t (relative energy norm) with A the 5-point stencil
of the state operator given beside the target and the free-node mask of the
input.
Training: Adam (Kingma and Ba, 2015) with beta1 = 0.9, beta2 = 0.999,
eps = 1e-8 and bias correction.

The bf16 helper rounds to the nearest bfloat16 (ties to even) so a test can
evaluate this network on the values the device network sees.

Flexible CG: Notay's FCG with truncation 1 (SIAM J. Sci. Comput. 22, 2000):
the new direction is the preconditioned residual A-orthogonalized against the
previous direction only, which admits a nonlinear preconditioner.
"""
from __future__ import annotations

import numpy as np

CHANNELS = 32
N_LAYERS = 6
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def layer_shapes(cin: int = 3, ch: int = CHANNELS, cout: int = 1):
    """[(c_out, c_in)] of the six convolutions."""
    return [(ch, cin)] + [(ch, ch)] * 4 + [(cout, ch)]


def n_params(shapes=None) -> int:
    shapes = shapes or layer_shapes()
    return sum(co * ci * 9 + co for co, ci in shapes)


def unpack(theta: np.ndarray, shapes=None):
    """Packed vector -> [(W (co, ci, 3, 3), b (co,))]; per layer W then b."""
    shapes = shapes or layer_shapes()
    out, o = [], 0
    for co, ci in shapes:
        W = theta[o:o + co * ci * 9].reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    assert o == theta.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def init_params(seed_gen: np.random.Generator, shapes=None, scale: float = 1.0) -> np.ndarray:
    """He-style normal init (std sqrt(2 / (9 c_in))), zero biases, last layer scaled by 0.1."""
    shapes = shapes or layer_shapes()
    layers = []
    for li, (co, ci) in enumerate(shapes):
        std = scale * np.sqrt(2.0 / (9.0 * ci)) * (0.1 if li == len(shapes) - 1 else 1.0)
        layers.append((std * seed_gen.standard_normal((co, ci, 3, 3)), np.zeros(co)))
    return pack(layers)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- conv ---
def conv(x, W, b=None):
    """x: (B, ci, H, Wd), W: (co, ci, 3, 3) -> (B, co, H, Wd), zero padding."""
    B, ci, H, Wd = x.shape
    xp = np.zeros((B, ci, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    y = np.zeros((B, W.shape[0], H, Wd))
    for a in range(3):
        for c in range(3):
            y += np.einsum("oc,bchw->bohw", W[:, :, a, c], xp[:, :, a:a + H, c:c + Wd])
    if b is not None:
        y += b[None, :, None, None]
    return y


def conv_backward(x, W, gy):
    """Gradients of sum(gy * conv(x, W, b)) w.r.t. x, W and b."""
    B, ci, H, Wd = x.shape
    xp = np.zeros((B, ci, H + 2, Wd + 2))
    xp[:, :, 1:-1, 1:-1] = x
    gW = np.zeros_like(W)
    gxp = np.zeros_like(xp)
    for a in range(3):
        for c in range(3):
            gW[:, :, a, c] = np.einsum("bohw,bchw->oc", gy, xp[:, :, a:a + H, c:c + Wd])
            gxp[:, :, a:a + H, c:c + Wd] += np.einsum("oc,bohw->bchw", W[:, :, a, c], gy)
    return gxp[:, :, 1:-1, 1:-1], gW, gy.sum(axis=(0, 2, 3))


# ------------------------------------------------------------- network ---
def forward(theta, x, round_bf16: bool = False, shapes=None):
    """Network output y (B, 1, H, W) and the cache of the backward pass.

    round_bf16: weights and every convolution input rounded to bf16 (the
    values the device network multiplies; sums stay exact here).  In the
    gradient the output gradient of every convolution is rounded likewise."""
    layers = unpack(np.asarray(theta, dtype=float), shapes)
    rnd = bf16 if round_bf16 else (lambda v: v)
    cache = []
    h = x
    for li, (W, b) in enumerate(layers):
        inp = rnd(h)
        z = conv(inp, rnd(W), b)
        cache.append((inp, z))
        if li == 0:
            h = np.maximum(z, 0.0)
        elif li < len(layers) - 1:
            h = h + np.maximum(z, 0.0)
        else:
            h = z
    return h, cache


def loss(y, t):
    """mean_b |y_b - t_b|^2 / |t_b|^2 and its gradient w.r.t. y."""
    B = y.shape[0]
    num = ((y - t) ** 2).reshape(B, -1).sum(axis=1)
    den = (t ** 2).reshape(B, -1).sum(axis=1)
    L = float(np.mean(num / den))
    gy = 2.0 * (y - t) / (den[:, None, None, None] * B)
    return L, gy


def stencil_apply(v, wE, wN, diag):
    """(A v) on an image: 5-point operator with edge weights wE (to the east
    neighbour), wN (to the north neighbour) and diagonal diag; neighbours
    outside the image count zero.  Arrays (..., H, W) indexed [row][column]."""
    Av = diag * v
    Av[..., :, :-1] -= wE[..., :, :-1] * v[..., :, 1:]
    Av[..., :, 1:] -= wE[..., :, :-1] * v[..., :, :-1]
    Av[..., :-1, :] -= wN[..., :-1, :] * v[..., 1:, :]
    Av[..., 1:, :] -= wN[..., :-1, :] * v[..., :-1, :]
    return Av


def energy_loss(y, t4, mask):
    """mean_b (d^T A d) / (t^T A t), d = (y - t) * mask, with A the 5-point
    stencil of t4[:, 1:4] = (wE, wN, diag); and its gradient w.r.t. y."""
    B = y.shape[0]
    t = t4[:, 0:1]
    wE, wN, dg = t4[:, 1:2], t4[:, 2:3], t4[:, 3:4]
    d = (y - t) * mask
    tm = t * mask
    Ad = stencil_apply(d, wE, wN, dg) * mask
    At = stencil_apply(tm, wE, wN, dg) * mask
    num = (d * Ad).reshape(B, -1).sum(axis=1)
    den = (tm * At).reshape(B, -1).sum(axis=1)
    L = float(np.mean(num / den))
    gy = 2.0 * Ad / (den[:, None, None, None] * B)
    return L, gy


def gradient(theta, x, t, round_bf16: bool = False, shapes=None):
    """Loss and its gradient (packed like theta).  t: (B, 1, H, W) for the
    relative L2 loss, (B, 4, H, W) = (target, wE, wN, diag) for the relative
    energy norm with the free-node mask taken from input channel 2."""
    layers = unpack(np.asarray(theta, dtype=float), shapes)
    rnd = bf16 if round_bf16 else (lambda v: v)
    y, cache = forward(theta, x, round_bf16, shapes)
    L, g = loss(y, t) if t.shape[1] == 1 else energy_loss(y, t, x[:, 2:3])
    grads = [None] * len(layers)
    # g holds dL/dh of the current layer's output
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        inp, z = cache[li]
        gz = rnd(g if li == len(layers) - 1 else g * (z > 0))
        gx, gW, gb = conv_backward(inp, rnd(W), gz)
        grads[li] = (gW, gb)
        if li > 0:
            # residual layers pass their output gradient straight through as well
            g = gx + (g if 0 < li < len(layers) - 1 else 0.0)
    return L, pack(grads)


def adam_step(theta, grad, m, v, step: int, lr: float):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = ADAM_B1 * m + (1.0 - ADAM_B1) * grad
    v = ADAM_B2 * v + (1.0 - ADAM_B2) * grad * grad
    mh = m / (1.0 - ADAM_B1 ** step)
    vh = v / (1.0 - ADAM_B2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v


# ---------------------------------------------------------- flexible CG ---
def fcg(A, b, prec, rtol: float = 1e-10, max_iter: int = 500, x0=None):
    """Flexible CG with truncation 1: solves A x = b (A SPD) with a possibly
    nonlinear preconditioner prec(r).  Returns (x, iterations, residual history)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - A(x)
    nb = np.linalg.norm(b)
    hist = [np.linalg.norm(r)]
    p_prev = q_prev = None
    it = 0
    while hist[-1] > rtol * nb and it < max_iter:
        z = prec(r)
        if p_prev is None:
            p = z
        else:
            p = z - (z @ q_prev) / (p_prev @ q_prev) * p_prev
        q = A(p)
        alpha = (p @ r) / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        p_prev, q_prev = p, q
        it += 1
        hist.append(np.linalg.norm(r))
    return x, it, hist
