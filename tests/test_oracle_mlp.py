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


def test_round_bf16_ties_to_even_and_nearest():
    r = mlp.round_bf16
    exact = np.array([1.0, 1.5, -2.0, 3.0, 0.0, 2.0 ** -20, -(1 + 2.0 ** -7)])
    assert np.array_equal(r(exact), exact)
    assert r(np.array([1 + 2.0 ** -8]))[0] == 1.0                       # tie -> even (1.0)
    assert r(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6         # tie -> even (1 + 2^-6)
    assert r(np.array([1 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1 + 2.0 ** -7
    assert r(np.array([-(1 + 2.0 ** -8 + 2.0 ** -20)]))[0] == -(1 + 2.0 ** -7)
    # brute force: the result has an 8-bit significand and no bf16 neighbour is closer
    x = (2 * synth.uniform(31, 2000) - 1) * 10.0 ** (8 * synth.uniform(32, 2000) - 4)
    y = r(x)
    bits = y.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)
    up = (bits.astype(np.uint64) + 0x10000).astype(np.uint32).view(np.float32).astype(np.float64)
    dn = (bits.astype(np.uint64) - 0x10000).astype(np.uint32).view(np.float32).astype(np.float64)
    xf = x.astype(np.float32).astype(np.float64)
    assert np.all(np.abs(xf - y) <= np.abs(xf - up)) and np.all(np.abs(xf - y) <= np.abs(xf - dn))


def test_bf16_operand_gradients_stay_close_to_exact():
    widths = [16, 32, 32, 8]
    params = mlp.init_params(widths, 5)
    X = 2 * synth.uniform(33, 40 * 16).reshape(40, 16) - 1
    Tg = synth.uniform(34, 40 * 8).reshape(40, 8)
    l0, g0 = mlp.loss_and_grads(params, X, Tg)
    l1, g1 = mlp.loss_and_grads(params, X, Tg, rnd=mlp.round_bf16)
    assert l1 != l0 and abs(l1 - l0) <= 2e-2 * l0
    for l in range(len(params)):
        for i in range(2):
            a, b = g1[l][i], g0[l][i]
            assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(b)
