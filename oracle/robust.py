"""Robust-satisfaction checks of a returned policy (the Monte-Carlo protocol of
the paper's methodology section, with the linearised closed form).

(i) Closed form: for each constraint the linearised worst case over the ball
    ||zeta|| <= r is g0_j + b_j' du + ||A_hat_j k_v + b_hat_j||, attained at
    zeta* = r c_j / ||c_j|| with c_j = eta_j / r.
(ii) Sampling with a fixed seed: uniform interior points of the ball
    (Gaussian direction by Box-Muller of SplitMix64 uniforms, radius
    r U^(1/d)), and "edge" points: convex combinations (Dirichlet(1) weights)
    of two or three worst-case directions zeta*_j, rescaled to ||zeta|| = r
    (a reading of the paper's edge-case construction).
Rollouts: linearised closed loop (must satisfy every constraint) and the
nonlinear closed loop u_k = u_hat_k + du_k + K_k zeta_k (a fraction is
reported).
"""
from __future__ import annotations

import numpy as np

import synth

from . import linearize, models


def worst_case(s, du, K):
    E = linearize.eta(s, K)
    return s.g0 + s.bmat @ du + np.sqrt(np.sum(E * E, axis=1))


def ball_samples(seed, n, d, r):
    u = synth.uniform(seed, 3 * n * d).reshape(3, n, d)
    z = np.sqrt(-2.0 * np.log(np.maximum(u[0], 1e-300))) * np.cos(2.0 * np.pi * u[1])
    z /= np.linalg.norm(z, axis=1, keepdims=True)
    rad = r * u[2, :, 0] ** (1.0 / d)
    return z * rad[:, None]


def edge_samples(seed, n, s, du, K):
    E = linearize.eta(s, K)
    nrm = np.linalg.norm(E, axis=1)
    dirs = E[nrm > 0] / nrm[nrm > 0, None]
    d = synth.Draws(seed)
    out = []
    for _ in range(n):
        m = int(d.ints(1, 2, 3)[0])
        idx = d.ints(m, 0, len(dirs) - 1)
        w = -np.log(np.maximum(d.u(m), 1e-300))
        w /= w.sum()
        v = (w[:, None] * dirs[idx]).sum(axis=0)
        nv = np.linalg.norm(v)
        if nv == 0:
            v = dirs[idx[0]]
            nv = 1.0
        out.append(s.radius * v / nv)
    return np.array(out)


def linear_rollout(s, du, K, zeta):
    T, nx, nu = s.T, s.nx, s.nu
    dx = np.zeros((T + 1, nx))
    dx[0] = zeta[:nx]
    dU = np.zeros((T, nu))
    for k in range(T):
        dU[k] = du[k * nu:(k + 1) * nu] + K[k] @ zeta[k * nx:(k + 1) * nx]
        dx[k + 1] = s.A[k] @ dx[k] + s.B[k] @ dU[k] + zeta[(k + 1) * nx:(k + 2) * nx]
    return dx, dU


def linear_constraints(s, dx, dU):
    out = np.empty(s.ng)
    for j in range(s.ng):
        if s.kind[j] == linearize.KIND_STATE:
            out[j] = s.g0[j] + s.w[j] @ dx[s.time[j]]
        else:
            out[j] = s.g0[j] + s.csign[j] * dU[s.time[j], s.cidx[j]]
    return out


def nonlinear_rollout(prob, u, K, zeta):
    T, nx = prob.T, prob.nx
    x = np.zeros((T + 1, nx))
    x[0] = prob.x0 + zeta[:nx]
    U = np.zeros((T, prob.nu))
    for k in range(T):
        U[k] = u[k] + K[k] @ zeta[k * nx:(k + 1) * nx]
        x[k + 1] = models.step(prob, x[k], U[k]) + zeta[(k + 1) * nx:(k + 2) * nx]
    return x, U
