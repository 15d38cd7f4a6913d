"""FP64 reference of the learned Newton initial guess (test infrastructure).

A multilayer perceptron 13 -> H -> H -> H -> 5 with SiLU activations maps
per-point features of the macroscopic state and velocity grid to the
correction of the Newton unknowns z over the cold guess (the continuous
equilibrium of the moments).  The paper solves the conservative-equilibrium
system by Newton (Section "Numerical method"); the network only supplies a
starting point, Newton alone decides convergence on the residual.

Flat parameter layout (shared with the GPU kernels through the C ABI, not
through code): for each layer [W (out x in, row major), b (out)], then the
5 output scales and 5 output offsets (z-score of the targets).
"""
from __future__ import annotations

import numpy as np

N_IN, N_OUT = 13, 5


def n_params(H: int) -> int:
    return H * N_IN + H + 2 * (H * H + H) + N_OUT * H + N_OUT + 2 * N_OUT


def layer_shapes(H: int):
    return [(H, N_IN), (H, H), (H, H), (N_OUT, H)]


def unpack(w: np.ndarray, H: int):
    w = np.asarray(w, np.float64)
    out, o = [], 0
    for (m, n) in layer_shapes(H):
        W = w[o:o + m * n].reshape(m, n)
        o += m * n
        b = w[o:o + m]
        o += m
        out.append((W, b))
    scale = w[o:o + N_OUT]
    offset = w[o + N_OUT:o + 2 * N_OUT]
    return out, scale, offset


def pack(layers, scale, offset) -> np.ndarray:
    parts = []
    for W, b in layers:
        parts += [np.asarray(W).reshape(-1), np.asarray(b).reshape(-1)]
    parts += [np.asarray(scale).reshape(-1), np.asarray(offset).reshape(-1)]
    return np.concatenate(parts)


def init(H: int, seed: int = 4) -> np.ndarray:
    """He-uniform weights, zero biases, unit output scale and zero offset."""
    rng = np.random.default_rng(seed)
    layers = []
    for (m, n) in layer_shapes(H):
        lim = np.sqrt(6.0 / n)
        layers.append((rng.uniform(-lim, lim, (m, n)), np.zeros(m)))
    return pack(layers, np.ones(N_OUT), np.zeros(N_OUT))


def silu(x):
    return x / (1.0 + np.exp(-x))


def dsilu(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def forward(w, X, H: int):
    """Network output y (normalised) for features X[B, 7]; also the cache of
    pre-activations for backpropagation."""
    layers, _, _ = unpack(w, H)
    a = np.asarray(X, np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        z = a @ W.T + b
        cache.append((a, z))
        a = z if li == len(layers) - 1 else silu(z)
    return a, cache


def predict(w, X, H: int):
    """Denormalised prediction dz = y * scale + offset."""
    y, _ = forward(w, X, H)
    _, scale, offset = unpack(w, H)
    return y * scale + offset


def loss_and_grad(w, X, T, H: int):
    """Mean squared error 1/(2B) sum |y - T|^2 on normalised targets T, and its
    gradient with respect to the network weights (output affine excluded:
    its gradient entries are zero)."""
    B = X.shape[0]
    y, cache = forward(w, X, H)
    layers, _, _ = unpack(w, H)
    r = y - T
    loss = 0.5 * np.sum(r * r) / B
    delta = r / B
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        a, z = cache[li]
        if li != len(layers) - 1:
            delta = delta * dsilu(z)
        W, _ = layers[li]
        grads.append((delta.T @ a, delta.sum(0)))
        delta = delta @ W
    grads = grads[::-1]
    return loss, pack(grads, np.zeros(N_OUT), np.zeros(N_OUT))


def adam_update(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on the flat vectors; returns new w, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def features(rho, U, theta, umax, nv):
    """Network inputs on the grid [-u_max, u_max]^3 with nv nodes per axis:
    [ln rho, U/u_max (3), ln theta, u_max/10, n_v/32, sin phi (3), cos phi (3)]
    with phi = 2 pi (U + u_max)/du, du = 2 u_max/(nv - 1): the trapezoid sum
    of a Gaussian differs from its integral by a Fourier series in this phase
    (Poisson summation)."""
    rho = np.asarray(rho, np.float64)
    U = np.asarray(U, np.float64)
    th = np.asarray(theta, np.float64)
    n = rho.shape[0]
    du = 2.0 * umax / (nv - 1)
    ph = 2.0 * np.pi * (U + umax) / du
    return np.concatenate([np.log(rho)[:, None], U / umax, np.log(th)[:, None],
                           np.full((n, 1), umax / 10.0), np.full((n, 1), nv / 32.0),
                           np.sin(ph), np.cos(ph)], 1)
