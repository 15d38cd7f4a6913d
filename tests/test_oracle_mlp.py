"""Pins of the FP64 MLP reference: backpropagation against central finite
differences, layout round trip, and the Adam formula on a quadratic."""
import numpy as np
import pytest

from oracle import mlp


def test_layout_and_count():
    # 13*64 + 64 + 2*(64*64 + 64) + 5*64 + 5 = 9541 network weights + output affine
    assert mlp.n_params(64) == 9541 + 10
    w = mlp.init(8, seed=1)
    layers, s, o = mlp.unpack(w, 8)
    assert np.array_equal(mlp.pack(layers, s, o), w)


def test_backprop_matches_central_differences():
    H = 6
    rng = np.random.default_rng(0)
    w = mlp.init(H, seed=2) + 0.1 * rng.standard_normal(mlp.n_params(H))
    X = rng.standard_normal((11, mlp.N_IN))
    T = rng.standard_normal((11, 5))
    loss, g = mlp.loss_and_grad(w, X, T, H)
    h = 1e-6
    nnet = mlp.n_params(H) - 10
    for i in rng.choice(nnet, 60, replace=False):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (mlp.loss_and_grad(wp, X, T, H)[0] - mlp.loss_and_grad(wm, X, T, H)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    assert np.all(g[nnet:] == 0)


def test_silu_derivative():
    x = np.linspace(-6, 6, 101)
    h = 1e-6
    assert np.allclose(mlp.dsilu(x), (mlp.silu(x + h) - mlp.silu(x - h)) / (2 * h), atol=1e-9)


def test_adam_minimises_quadratic():
    w = np.array([3.0, -2.0])
    m = v = np.zeros(2)
    for t in range(1, 3001):
        w, m, v = mlp.adam_update(w, 2 * w, m, v, t, 0.05)
    assert np.abs(w).max() < 1e-3


def test_grid_phase_feature_governs_trapezoid_aliasing():
    """The phase features are those of the Poisson-summation error of the
    trapezoid rule: on nodes -u_max + k du the sum of a unit 1-D Gaussian of
    variance theta is 1 + 2 exp(-2 pi^2 theta/du^2) cos(phi) + O(exp(-8 pi^2
    theta/du^2)), phi = 2 pi (U + u_max)/du."""
    umax, nv = 10.0, 21
    du = 2 * umax / (nv - 1)
    u = -umax + du * np.arange(nv)
    w = np.full(nv, du)
    w[0] = w[-1] = du / 2
    rng = np.random.default_rng(3)
    for _ in range(20):
        U = rng.uniform(-2, 2)
        th = rng.uniform(0.06, 0.12)
        g = np.exp(-(u - U) ** 2 / (2 * th)) / np.sqrt(2 * np.pi * th)
        x = mlp.features(np.ones(1), np.array([[U, 0.0, 0.0]]), np.array([th]), umax, nv)[0]
        a = np.exp(-2 * np.pi ** 2 * th / du ** 2)
        assert abs((w @ g - 1.0) - 2 * a * x[10]) <= 4 * a ** 4 + 1e-13
        assert abs(x[7] ** 2 + x[10] ** 2 - 1.0) < 1e-12
