"""FP64 reference of the warm-start network (a learned warm start is the
paper's stated future work; the network here maps problem parameters to the
NRTO-DR primal/dual iterates).

Architecture: widths w_0 -> w_1 -> ... -> w_L, affine layers z = a W' + b,
GELU x Phi(x) (exact, with erf) after every layer but the last.  Loss: mean
squared error over batch and outputs, L = sum (y - t)^2 / (B * D).  Adam
(Kingma and Ba 2015): m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
theta -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
Initial weights uniform in +-sqrt(6 / (fan_in + fan_out)) from SplitMix64,
biases zero.  forward / loss_and_grads optionally round every GEMM operand
(round_bf16: bfloat16, round to nearest even) to model matrix-core products
of bfloat16 operands; the arithmetic between rounding points stays FP64.
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


def round_bf16(x):
    """x rounded to the nearest bfloat16 value (ties to even), as float64: the
    float32 value of x keeps its top 16 bits after adding half an ulp of the
    16-bit result (IEEE round-to-nearest-even on an 8-bit significand)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(params, X, rnd=None):
    """rnd: None (exact FP64) or a rounding applied to every GEMM operand (the
    layer inputs and the weights), as the matrix cores see them."""
    q = (lambda v: v) if rnd is None else rnd
    acts = [q(X)]
    pre = []
    a = acts[0]
    for l, (W, b) in enumerate(params):
        z = a @ q(W).T + b
        pre.append(z)
        if l < len(params) - 1:
            a = q(gelu(z))
        else:
            a = z
        acts.append(a)
    return a, acts, pre


def loss_and_grads(params, X, Tgt, rnd=None):
    """Loss and gradients; with rnd, the backward GEMM operands (the output
    gradient of each layer and the weights) are rounded too, while the bias
    gradients sum the unrounded output gradients."""
    q = (lambda v: v) if rnd is None else rnd
    Y, acts, pre = forward(params, X, rnd)
    B, D = Y.shape
    diff = Y - Tgt
    loss = float(np.sum(diff * diff) / (B * D))
    g = 2.0 * diff / (B * D)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        if l < len(params) - 1:
            g = g * gelu_grad(pre[l])
        gq = q(g)
        grads[l] = [gq.T @ acts[l], g.sum(axis=0)]
        g = gq @ q(W)
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
