"""Pins of the MLP oracle: central finite differences, a textbook GELU, Adam."""

import math

import numpy as np
import pytest

from oracle import mlp


def test_param_count():
    assert mlp.n_params() == 148995


def test_gelu_against_textbook_values():
    # Phi(1) = 0.841344746..., Phi(-1) = 0.158655254..., gelu(0) = 0
    np.testing.assert_allclose(mlp.gelu(np.array([1.0, -1.0, 0.0])),
                               [0.8413447460685429, -0.15865525393145707, 0.0], rtol=1e-14)
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), rtol=1e-8,
                               atol=1e-10)


def test_backward_matches_central_differences():
    r = np.random.default_rng(0)
    theta = mlp.init_params(1)
    X = r.standard_normal((5, 64))
    T = r.standard_normal((5, 3))
    g, _ = mlp.backward(theta, X, T)
    idx = np.concatenate([r.choice(mlp.n_params(), 60, replace=False),
                          [0, 16383, 16384, 16639, mlp.n_params() - 1, mlp.n_params() - 4]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, T) - mlp.loss(tm, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_bf16_round():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.14159])
    y = mlp.bf16_round(x)
    assert y[0] == 1.0 and y[1] == 1.0  # tie to even
    assert y[2] == 1.0 + 2 ** -7
    assert y[3] == -2.5
    assert abs(y[4] - 3.14159) <= 2 ** -8 * 4


def test_adam_first_step_is_signed_lr():
    theta = np.zeros(4)
    g = np.array([1.0, -2.0, 0.5, 0.0])
    t, m, v = mlp.adam_step(theta, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(t[:3], -0.01 * np.sign(g[:3]), rtol=1e-6)
    assert t[3] == 0.0
