"""FP64 oracle of the surrogate network (test infrastructure only).

The surrogate of logL(theta) is an ensemble of small fully connected
networks, n_in -> H -> H -> 1 with GELU after each hidden layer, trained by
mean-squared error with Adam. This module is a plain numpy FP64 statement of
the forward pass, the hand-derived backward pass, one Adam step, the ensemble
mean/spread and the gate rule. It imports nothing from the product package.

Parameter layout of one member (flat, row-major matrices):
    W1 [H, n_in], b1 [H], W2 [H, H], b2 [H], W3 [H] (the 1 x H output row), b3 [1]
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def n_params(n_in: int, H: int) -> int:
    return H * n_in + H + H * H + H + H + 1


def unpack(p: np.ndarray, n_in: int, H: int):
    o = 0
    W1 = p[o:o + H * n_in].reshape(H, n_in); o += H * n_in
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o:o + 1]; o += 1
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def gelu(x):
    """Exact GELU: x Phi(x) = x (1 + erf(x / sqrt 2)) / 2."""
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(p, x, n_in, H):
    """Network output f[N] for inputs x[N, n_in], plus the cache for backward."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, H)
    z1 = x @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    f = h2 @ W3 + b3[0]
    return f, (x, z1, h1, z2, h2)


def loss_and_grad(p, x, y, n_in, H):
    """Mean squared error L = mean_s (f_s - y_s)^2 and dL/dp, by the chain
    rule written out layer by layer."""
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, H)
    f, (x, z1, h1, z2, h2) = forward(p, x, n_in, H)
    N = x.shape[0]
    r = f - y
    loss = float(np.mean(r * r))
    df = 2.0 * r / N                       # dL/df
    gW3 = h2.T @ df
    gb3 = np.array([df.sum()])
    dz2 = (df[:, None] * W3[None, :]) * gelu_grad(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, gb3])
    return loss, g


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected moments), returning new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def he_init(rng, n_in, H):
    """He-normal weights N(0, 2/fan_in), zero biases."""
    W1 = rng.standard_normal((H, n_in)) * math.sqrt(2.0 / n_in)
    W2 = rng.standard_normal((H, H)) * math.sqrt(2.0 / H)
    W3 = rng.standard_normal(H) * math.sqrt(2.0 / H)
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3, np.zeros(1)])


def scale_inputs(theta, lo, hi):
    """Prior box [lo, hi] -> [-1, 1]."""
    return 2.0 * (np.asarray(theta) - lo) / (hi - lo) - 1.0


def ensemble(params, theta, lo, hi, y_mean, y_std, n_in, H):
    """Mean and population spread (ddof = 0) of the members' predictions in
    logL units."""
    x = scale_inputs(theta, lo, hi)
    preds = np.stack([y_mean + y_std * forward(p, x, n_in, H)[0] for p in params])
    return preds.mean(axis=0), preds.std(axis=0, ddof=0)


def gate(mean, spread, L_min, tau):
    """1 = evaluate exactly, 0 = reject without an exact call.
    Spread above tau falls back to the exact likelihood; a confident
    prediction below the current threshold is rejected; a confident
    prediction above it is still judged exactly."""
    mean = np.asarray(mean)
    spread = np.asarray(spread)
    reject = (spread <= tau) & (mean < L_min)
    return np.where(reject, 0, 1).astype(np.int32)
