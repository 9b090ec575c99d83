"""Pins of the FP64 reference network of the learned order predictor (CPU)."""
import math

import numpy as np

from oracle import mlp


def test_gelu_textbook_values_and_derivative():
    # gelu(x) = x Phi(x); Phi(1) = 0.841344746068543, Phi(-2) = 0.0227501319481792
    assert abs(mlp.gelu(np.array(1.0)) - 0.841344746068543) < 1e-14
    assert abs(mlp.gelu(np.array(-2.0)) - (-2.0 * 0.0227501319481792)) < 1e-14
    x = np.linspace(-4, 4, 33)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-8


def test_zero_network_gives_uniform_loss():
    theta = np.zeros(mlp.NPARAMS)
    x = np.random.default_rng(0).standard_normal((7, 32))
    loss, g = mlp.loss_and_grad(theta, x, [0, 1, 2, 3, 4, 0, 1])
    assert abs(loss - math.log(5.0)) < 1e-14
    assert mlp.NPARAMS == 21381


def test_gradient_matches_central_differences():
    g = np.random.default_rng(1)
    theta = g.standard_normal(mlp.NPARAMS) * 0.2
    x = g.standard_normal((6, 32))
    y = g.integers(0, 5, 6)
    loss, grad = mlp.loss_and_grad(theta, x, y)
    idx = np.concatenate([g.choice(mlp.NPARAMS, 60, replace=False), [21376, 21380, 0, 4096, 4224, 20608, 20736]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, x, y)[0] - mlp.loss_and_grad(tm, x, y)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 + 1e-6 * abs(fd)


def test_features_invariances():
    g = np.random.default_rng(2)
    mt = g.standard_normal(8) + 1j * g.standard_normal(8)
    f = mlp.features(mt, 3.0)
    # a global phase of the bin and the bin's scale (apart from f[24]) do not change the features
    f2 = mlp.features(mt * np.exp(1.3j) * 7.0, 3.0)
    assert np.allclose(f[:24], f2[:24], atol=1e-12)
    assert abs(f2[24] - f[24] - math.log(49.0)) < 1e-12
    assert abs(f[1]) < 1e-15 and f[0] > 0          # u_0 is real and positive
    assert abs(np.sum(f[16:24] ** 2) - 8.0) < 1e-12   # magnitudes normalised to mean square 1
    assert np.all(f[25:] == 0)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7 + 2 ** -9, -3.1415926])
    r = mlp.bf16_round(v)
    assert r[0] == 1.0 and r[1] == 1.0                 # tie to even
    assert r[2] == 1.0 + 2 ** -7                      # below half an ulp: rounds down
    assert abs(r[3] + 3.140625) < 1e-12


def test_backward_rounding_points_bound():
    """bf16_backward rounds the deltas dZ3 (for the W3 side), dZ2 and dZ1 to
    bfloat16 (relative error at most 2^-9 each).  The rounded gradient then
    differs from the unrounded one of the same (BF16-forward) network by at
    most the first-order propagation of those errors, bounded entry by entry
    through the absolute values of the factors; b3 is untouched."""
    g = np.random.default_rng(4)
    theta = g.standard_normal(mlp.NPARAMS) * 0.2
    x = g.standard_normal((40, 32))
    y = g.integers(0, 5, 40)
    _, g0 = mlp.loss_and_grad(theta, x, y, bf16=True)
    _, g1 = mlp.loss_and_grad(theta, x, y, bf16=True, bf16_backward=True)
    p0, p1 = mlp.unpack(g0), mlp.unpack(g1)
    assert np.array_equal(p0["b3"], p1["b3"])
    for name in ("W3", "W2", "W1", "b2", "b1"):
        rel = np.max(np.abs(p1[name] - p0[name])) / np.max(np.abs(p0[name]))
        # one rounding on each delta layer between the loss and the parameter:
        # W3: 1, W2/b2: 2, W1/b1: 3 roundings of at most 2^-9, summed in |.|
        assert 0 < rel < 3 * 2.0 ** -9 * 40, (name, rel)
    # zero deltas round to zero: a network with zero last layer has dZ2 = dZ1 = 0
    t0 = theta.copy()
    t0[mlp.NPARAMS - 5 - 5 * 128:mlp.NPARAMS - 5] = 0.0
    _, ga = mlp.loss_and_grad(t0, x, y, bf16=True)
    _, gb = mlp.loss_and_grad(t0, x, y, bf16=True, bf16_backward=True)
    pa, pb = mlp.unpack(ga), mlp.unpack(gb)
    assert np.all(pb["W1"] == 0) and np.all(pb["W2"] == 0) and np.all(pa["W1"] == 0)
