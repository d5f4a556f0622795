"""FP64 reference of the warm-start network (a learned warm start is the
paper's stated future work; the network here maps problem parameters to the
NRTO-DR primal/dual iterates).

Architecture: widths w_0 -> w_1 -> ... -> w_L, affine layers z = a W' + b,
GELU x Phi(x) (exact, with erf) after every layer but the last.  Loss: mean
squared error over batch and outputs, L = sum (y - t)^2 / (B * D).  Adam
(Kingma and Ba 2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
Initial weights uniform in +-sqrt(6 / (fan_in + fan_out)) from SplitMix64,
biases zero.
"""
from __future__ import annotations

import math

import numpy as np

import synth


def init_params(widths, seed):
    params = []
    for l in range(len(widths) - 1):
        fi, fo = widths[l], widths[l + 1]
        a = math.sqrt(6.0 / (fi + fo))
        W = (2.0 * synth.uniform(synth.stream_seed(seed, l), fo * fi) - 1.0).reshape(fo, fi) * a
        params.append([W, np.zeros(fo)])
    return params


def gelu(x):
    from scipy.special import erf
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(params, X):
    acts = [X]
    pre = []
    a = X
    for l, (W, b) in enumerate(params):
        z = a @ W.T + b
        pre.append(z)
        a = gelu(z) if l < len(params) - 1 else z
        acts.append(a)
    return a, acts, pre


def loss_and_grads(params, X, Tgt):
    Y, acts, pre = forward(params, X)
    B, D = Y.shape
    diff = Y - Tgt
    loss = float(np.sum(diff * diff) / (B * D))
    g = 2.0 * diff / (B * D)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        if l < len(params) - 1:
            g = g * gelu_grad(pre[l])
        grads[l] = [g.T @ acts[l], g.sum(axis=0)]
        g = g @ W
    return loss, grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [[np.zeros_like(p) for p in layer] for layer in params]
        self.v = [[np.zeros_like(p) for p in layer] for layer in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        for l in range(len(params)):
            for i in range(2):
                g = grads[l][i]
                self.m[l][i] = self.b1 * self.m[l][i] + (1 - self.b1) * g
                self.v[l][i] = self.b2 * self.v[l][i] + (1 - self.b2) * g * g
                mh = self.m[l][i] / (1 - self.b1 ** self.t)
                vh = self.v[l][i] / (1 - self.b2 ** self.t)
                params[l][i] = params[l][i] - self.lr * mh / (np.sqrt(vh) + self.eps)
