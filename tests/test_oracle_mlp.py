"""Pins of the FP64 reference MLP: central finite differences of the loss for
every parameter tensor, the closed-form GELU values Phi(0) = 1/2 and the
derivative, and one Adam step against its definition."""
import math

import numpy as np

import synth
from oracle import mlp


def test_gelu_values():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    x = np.linspace(-4, 4, 41)
    fd = (mlp.gelu(x + 1e-6) - mlp.gelu(x - 1e-6)) / 2e-6
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-8


def test_gradients_match_finite_differences():
    widths = [5, 7, 6, 4]
    params = mlp.init_params(widths, 3)
    for l in range(len(params)):
        params[l][1] = 0.1 * (2 * synth.uniform(100 + l, params[l][1].size) - 1)
    X = 2 * synth.uniform(1, 9 * 5).reshape(9, 5) - 1
    Tg = synth.uniform(2, 9 * 4).reshape(9, 4)
    _, grads = mlp.loss_and_grads(params, X, Tg)
    h = 1e-6
    for l in range(len(params)):
        for i in range(2):
            P = params[l][i]
            G = grads[l][i]
            flat = P.reshape(-1)
            for idx in range(0, flat.size, max(1, flat.size // 7)):
                old = flat[idx]
                flat[idx] = old + h
                lp, _ = mlp.loss_and_grads(params, X, Tg)
                flat[idx] = old - h
                lm, _ = mlp.loss_and_grads(params, X, Tg)
                flat[idx] = old
                assert abs((lp - lm) / (2 * h) - G.reshape(-1)[idx]) <= 1e-8


def test_adam_first_step_is_signed_lr():
    # with zero state the bias-corrected first step is lr * g / (|g| + eps)
    params = [[np.array([[1.0, -2.0]]), np.array([0.5])]]
    grads = [[np.array([[0.3, -0.4]]), np.array([2.0])]]
    opt = mlp.Adam(params, lr=0.01)
    opt.step(params, grads)
    assert np.allclose(params[0][0], [[1.0 - 0.01 * 0.3 / (0.3 + 1e-8), -2.0 + 0.01 * 0.4 / (0.4 + 1e-8)]])
    assert np.allclose(params[0][1], [0.5 - 0.01 * 2.0 / (2.0 + 1e-8)])
