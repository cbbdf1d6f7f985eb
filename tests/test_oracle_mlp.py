"""Pins of the FP64 surrogate-network oracle: finite differences of its own
loss, torch autograd as an independent derivative, closed forms of GELU and
of the first Adam step."""
import math

import numpy as np
import pytest

from oracle import mlp


def _problem(seed=0, n_in=5, H=7, N=13):
    rng = np.random.default_rng(seed)
    p = mlp.he_init(rng, n_in, H)
    p[n_in * H:n_in * H + H] = rng.standard_normal(H) * 0.1     # nonzero b1
    x = rng.uniform(-1, 1, size=(N, n_in))
    y = rng.standard_normal(N)
    return p, x, y, n_in, H


def test_param_count():
    assert mlp.n_params(12, 256) == 69377


def test_gelu_values():
    # GELU(0) = 0, GELU(x) -> x for large x, GELU(-x) = GELU(x) - x
    x = np.array([-3.0, -1.0, 0.0, 0.5, 2.0, 8.0])
    g = mlp.gelu(x)
    assert g[2] == 0.0
    np.testing.assert_allclose(mlp.gelu(-x), g - x, atol=1e-15)
    assert abs(g[-1] - 8.0) < 1e-12
    # x Phi(x) with Phi from math.erfc at one point
    assert abs(g[4] - 2.0 * 0.5 * math.erfc(-2.0 / math.sqrt(2))) < 1e-15


def test_gelu_grad_finite_difference():
    x = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, atol=1e-9)


def test_gradient_central_differences():
    p, x, y, n_in, H = _problem()
    _, g = mlp.loss_and_grad(p, x, y, n_in, H)
    fd = np.empty_like(p)
    for i in range(p.size):
        h = 1e-6 * max(1.0, abs(p[i]))
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd[i] = (mlp.loss_and_grad(pp, x, y, n_in, H)[0] - mlp.loss_and_grad(pm, x, y, n_in, H)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    p, x, y, n_in, H = _problem(seed=1, n_in=12, H=32, N=40)
    _, g = mlp.loss_and_grad(p, x, y, n_in, H)
    tp = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    o = 0
    W1 = tp[o:o + H * n_in].view(H, n_in); o += H * n_in
    b1 = tp[o:o + H]; o += H
    W2 = tp[o:o + H * H].view(H, H); o += H * H
    b2 = tp[o:o + H]; o += H
    W3 = tp[o:o + H]; o += H
    b3 = tp[o:o + 1]
    tx = torch.tensor(x)
    h1 = torch.nn.functional.gelu(tx @ W1.T + b1)
    h2 = torch.nn.functional.gelu(h1 @ W2.T + b2)
    f = h2 @ W3 + b3
    loss = ((f - torch.tensor(y)) ** 2).mean()
    loss.backward()
    np.testing.assert_allclose(g, tp.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_first_adam_step_closed_form():
    # From zero moments, bias correction makes the first step lr*g/(|g|+eps).
    g = np.array([3.0, -0.2, 1e-3, 0.0])
    p = np.zeros(4)
    p1, m, v = mlp.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-8)
    np.testing.assert_allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    p, x, y, n_in, H = _problem(seed=2, n_in=3, H=16, N=64)
    y = np.sin(2 * x[:, 0]) + x[:, 1] * x[:, 2]
    m = np.zeros_like(p); v = np.zeros_like(p)
    l0 = mlp.loss_and_grad(p, x, y, n_in, H)[0]
    for t in range(1, 301):
        _, g = mlp.loss_and_grad(p, x, y, n_in, H)
        p, m, v = mlp.adam_step(p, g, m, v, t, lr=1e-2)
    assert mlp.loss_and_grad(p, x, y, n_in, H)[0] < 0.05 * l0


def test_ensemble_spread_and_gate():
    rng = np.random.default_rng(3)
    n_in, H = 2, 4
    params = [mlp.he_init(rng, n_in, H) for _ in range(5)]
    th = rng.uniform(-1, 3, size=(6, n_in))
    mu, s = mlp.ensemble(params, th, -1.0, 3.0, 10.0, 2.0, n_in, H)
    preds = np.stack([10.0 + 2.0 * mlp.forward(p, mlp.scale_inputs(th, -1, 3), n_in, H)[0] for p in params])
    np.testing.assert_allclose(s, np.sqrt(((preds - preds.mean(0)) ** 2).mean(0)), rtol=1e-12)
    dec = mlp.gate(np.array([1.0, 1.0, 5.0, 5.0]), np.array([0.01, 0.2, 0.01, 0.2]), 3.0, 0.05)
    np.testing.assert_array_equal(dec, [0, 1, 1, 1])


def test_scale_inputs_fixed_points():
    """The prior box maps onto [-1, 1] input by input (reading of the
    surrogate's inputs): each lower edge goes to -1, each upper edge to +1,
    the midpoint to 0 and the three-quarter point to 0.5, with a box of its
    own per input. These four points fix an affine map per input."""
    lo = np.array([-1.0, 0.0, 2.0, -5.0])
    hi = np.array([3.0, 10.0, 2.5, -4.0])
    np.testing.assert_array_equal(mlp.scale_inputs(lo[None, :], lo, hi), [[-1.0] * 4])
    np.testing.assert_array_equal(mlp.scale_inputs(hi[None, :], lo, hi), [[1.0] * 4])
    np.testing.assert_allclose(mlp.scale_inputs(((lo + hi) / 2)[None, :], lo, hi), [[0.0] * 4], atol=1e-15)
    np.testing.assert_allclose(mlp.scale_inputs((lo + 0.75 * (hi - lo))[None, :], lo, hi), [[0.5] * 4],
                               atol=1e-15)
    # a row mixing edges of different inputs
    th = np.array([[3.0, 0.0, 2.25, -5.0]])
    np.testing.assert_allclose(mlp.scale_inputs(th, lo, hi), [[1.0, -1.0, 0.0, -1.0]], atol=1e-15)


def _constant_member(n_in, H, value):
    """A member whose output is `value` for every input: every weight zero
    and the output bias set."""
    p = np.zeros(mlp.n_params(n_in, H))
    p[-1] = value
    return p


def test_ensemble_destandardisation_constant_members():
    """Targets are standardised for training, so a member's output f stands
    for y_mean + y_std f in logL units (reading of the surrogate's targets),
    and the spread is the population standard deviation (ddof = 0) of the
    members in those units. Members with constant outputs fix both."""
    n_in, H = 3, 5
    th = np.array([[-1.0, 0.0, 3.0], [2.0, 2.0, 2.0], [0.5, -0.5, 1.5]])
    y_mean, y_std = -58000.0, 250.0
    # identical members: mean = y_mean + y_std f, spread exactly 0
    params = [_constant_member(n_in, H, 0.4)] * 5
    mu, s = mlp.ensemble(params, th, -1.0, 3.0, y_mean, y_std, n_in, H)
    np.testing.assert_allclose(mu, y_mean + y_std * 0.4, rtol=1e-15)
    np.testing.assert_array_equal(s, 0.0)
    # outputs (-1, 1, -1, 1, 0) a: mean y_mean, spread y_std a sqrt(4/5)
    a = 0.02
    params = [_constant_member(n_in, H, v * a) for v in (-1.0, 1.0, -1.0, 1.0, 0.0)]
    mu, s = mlp.ensemble(params, th, -1.0, 3.0, y_mean, y_std, n_in, H)
    np.testing.assert_allclose(mu, y_mean, rtol=1e-15)
    np.testing.assert_allclose(s, y_std * a * math.sqrt(0.8), rtol=1e-12)
    # the gate reads the spread in logL units: 0.05 * 250 = 12.5 > tau
    assert np.all(mlp.gate(mu - 100.0, s, y_mean, 0.05) == 1)
    assert np.all(mlp.gate(mu - 100.0, s / (y_std * a * 100.0), y_mean, 0.05) == 0)
