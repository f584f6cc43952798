"""FP64 reference of the warm-start network.  TEST INFRASTRUCTURE ONLY.

A fully connected network with GELU (exact erf form) after every layer but
the last, mean squared error loss, and Adam (Kingma & Ba) -- plain numpy in
double precision, written from the definitions: no fusion, no reordering.
Parameters are packed per layer l as W_l [n_l][n_{l+1}] (y = x W + b) then
b_l [n_{l+1}], the same packing as the library's iblb_mlp_* calls.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def unpack(params, widths):
    out, o = [], 0
    for l in range(len(widths) - 1):
        n_in, n_out = widths[l], widths[l + 1]
        W = params[o:o + n_in * n_out].reshape(n_in, n_out)
        o += n_in * n_out
        b = params[o:o + n_out]
        o += n_out
        out.append((W, b))
    assert o == len(params)
    return out


def param_count(widths):
    return sum(widths[l] * widths[l + 1] + widths[l + 1] for l in range(len(widths) - 1))


def init_params(widths, seed):
    """Seeded initial weights (uniform +-1/sqrt(fan_in), zero biases)."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(widths) - 1):
        bound = 1.0 / math.sqrt(widths[l])
        parts.append(rng.uniform(-bound, bound, size=widths[l] * widths[l + 1]))
        parts.append(np.zeros(widths[l + 1]))
    return np.concatenate(parts)


def forward(params, widths, x):
    """Returns the output and the per-layer (input, pre-activation) pairs."""
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    h = np.asarray(x, dtype=np.float64)
    cache = []
    for l, (W, b) in enumerate(layers):
        z = h @ W + b
        cache.append((h, z))
        h = gelu(z) if l < len(layers) - 1 else z
    return h, cache


def loss_and_grad(params, widths, x, t):
    """Mean squared error over all outputs and its gradient (packed)."""
    y, cache = forward(params, widths, x)
    t = np.asarray(t, dtype=np.float64)
    n = y.size
    loss = float(np.sum((y - t) ** 2) / n)
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    dz = 2.0 * (y - t) / n
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        h, _ = cache[l]
        W, _ = layers[l]
        dW = h.T @ dz
        db = dz.sum(axis=0)
        grads[l] = (dW, db)
        if l > 0:
            dh = dz @ W.T
            dz = dh * gelu_grad(cache[l - 1][1])
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


class Adam:
    def __init__(self, n, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = beta1, beta2, eps

    def step(self, params, grad, lr):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * grad
        self.v = self.b2 * self.v + (1 - self.b2) * grad * grad
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return params - lr * mh / (np.sqrt(vh) + self.eps)
