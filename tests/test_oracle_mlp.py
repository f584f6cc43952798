"""Pins of the FP64 reference network: GELU against its definition's
special values and derivative, gradients against central finite
differences, Adam's first step against its closed form."""
import math

import numpy as np

from oracle import mlp


def test_gelu_values_and_derivative():
    z = np.linspace(-6, 6, 241)
    g = mlp.gelu(z)
    assert abs(mlp.gelu(np.array([0.0]))[0]) == 0.0
    assert np.allclose(g[z > 5], z[z > 5], atol=1e-6)       # -> identity
    assert np.allclose(g[z < -5], 0.0, atol=1e-5)           # -> zero
    # GELU(z) - GELU(-z) = z (Phi(z) + Phi(-z) = 1)
    assert np.allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-8)


def test_gradient_matches_finite_differences():
    widths = [4, 7, 6, 5]
    rng = np.random.default_rng(0)
    p = mlp.init_params(widths, 1) + 0.05 * rng.standard_normal(mlp.param_count(widths))
    x = rng.standard_normal((9, 4))
    t = rng.standard_normal((9, 5))
    _, g = mlp.loss_and_grad(p, widths, x, t)
    h = 1e-6
    for i in range(len(p)):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, widths, x, t)[0] - mlp.loss_and_grad(pm, widths, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_linear_network_is_least_squares():
    """One linear layer: the gradient vanishes at the least-squares fit."""
    rng = np.random.default_rng(2)
    x = rng.standard_normal((50, 3))
    t = rng.standard_normal((50, 2))
    X1 = np.hstack([x, np.ones((50, 1))])
    sol = np.linalg.lstsq(X1, t, rcond=None)[0]
    p = np.concatenate([sol[:3].ravel(), sol[3]])
    _, g = mlp.loss_and_grad(p, [3, 2], x, t)
    assert np.max(np.abs(g)) < 1e-12


def test_adam_first_step_is_signed_lr():
    a = mlp.Adam(3)
    p = np.zeros(3)
    g = np.array([0.3, -2.0, 1e-3])
    q = a.step(p, g, 0.01)
    # after one step m_hat = g, v_hat = g^2: the update is lr * sign(g)
    assert np.allclose(q, -0.01 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), atol=1e-12)
