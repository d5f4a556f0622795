"""Pins of the oracle's robust constraint data (supplementary section I):
F_u and F_zeta against finite differences of the nonlinear rollout with
disturbances, the closed-form worst case against the linearised closed-loop
rollout at the maximiser and against sampling of the ball, the structured
operators against A_hat_j written out from its definition, and the support
of each cone (the compaction the GPU layout relies on)."""
import numpy as np
import pytest

import synth
from oracle import linearize, models


def _rollout_dist(prob, u, zeta):
    T, nx = prob.T, prob.nx
    x = np.zeros((T + 1, nx))
    x[0] = prob.x0 + zeta[:nx]
    for k in range(T):
        x[k + 1] = models.step(prob, x[k], u[k]) + zeta[(k + 1) * nx:(k + 2) * nx]
    return x


def _small(make, T):
    prob = make()
    prob.T = T
    prob.u_init = prob.u_init[:T]
    return prob


@pytest.mark.parametrize("make,T", [(synth.config1, 6), (synth.config2, 5), (synth.config3, 4)])
def test_sensitivities_match_finite_differences(make, T):
    prob = _small(make, T)
    d = synth.Draws(3)
    u = prob.u_init + d.u(T * prob.nu, -0.3, 0.3).reshape(T, prob.nu)
    s = linearize.assemble(prob, u)
    nz = (T + 1) * prob.nx
    h = 1e-6
    for k in range(T * prob.nu):
        e = np.zeros(T * prob.nu)
        e[k] = h
        xp = linearize.rollout(prob, u + e.reshape(T, -1))
        xm = linearize.rollout(prob, u - e.reshape(T, -1))
        assert np.allclose((xp - xm).ravel() / (2 * h), s.Fu[:, k], atol=1e-7)
    for i in range(nz):
        z = np.zeros(nz)
        z[i] = h
        fd = (_rollout_dist(prob, u, z) - _rollout_dist(prob, u, -z)).ravel() / (2 * h)
        assert np.allclose(fd, s.Fz[:, i], atol=1e-7)


def _lin_closed_loop(s, du, K, zeta):
    """Linearised closed-loop deviations with u_k = u_hat_k + du_k + K_k zeta_k."""
    T, nx, nu = s.T, s.nx, s.nu
    dx = np.zeros((T + 1, nx))
    dx[0] = zeta[:nx]
    dU = np.zeros((T, nu))
    for k in range(T):
        dU[k] = du[k * nu:(k + 1) * nu] + K[k] @ zeta[k * nx:(k + 1) * nx]
        dx[k + 1] = s.A[k] @ dx[k] + s.B[k] @ dU[k] + zeta[(k + 1) * nx:(k + 2) * nx]
    return dx, dU


def _lin_constraint(s, j, dx, dU):
    if s.kind[j] == linearize.KIND_STATE:
        return s.g0[j] + s.w[j] @ dx[s.time[j]]
    k, i, sg = s.time[j], s.cidx[j], s.csign[j]
    return s.g0[j] + sg * dU[k, i]


@pytest.mark.parametrize("make,T", [(synth.config1, 8), (synth.config2, 6)])
def test_worst_case_closed_form(make, T):
    prob = _small(make, T)
    s = linearize.assemble(prob, prob.u_init)
    d = synth.Draws(7)
    du = d.u(T * s.nu, -0.2, 0.2)
    K = d.u(T * s.nu * s.nx, -0.5, 0.5).reshape(T, s.nu, s.nx)
    E = linearize.eta(s, K)
    r = s.radius
    nz = s.nz
    samples = d.u(200 * nz, -1.0, 1.0).reshape(200, nz)
    for j in range(s.ng):
        worst = s.g0[j] + s.bmat[j] @ du + np.linalg.norm(E[j])
        c = E[j] / r                       # the linear functional of zeta
        if np.linalg.norm(c) == 0:
            continue
        zs = r * c / np.linalg.norm(c)
        dx, dU = _lin_closed_loop(s, du, K, zs)
        assert _lin_constraint(s, j, dx, dU) == pytest.approx(worst, abs=1e-10)
        for zz in samples[:40]:
            zz = zz * (r / np.linalg.norm(zz)) * 0.999
            dx, dU = _lin_closed_loop(s, du, K, zz)
            assert _lin_constraint(s, j, dx, dU) <= worst + 1e-12


def test_structured_operators_match_definition():
    prob = _small(synth.config2, 4)
    s = linearize.assemble(prob, prob.u_init)
    d = synth.Draws(8)
    kv = d.u(s.T * s.nu * s.nx, -1, 1)
    K = linearize.kv_to_K(kv, s.T, s.nu, s.nx)
    assert np.allclose(linearize.K_to_kv(K), kv)
    E = linearize.eta(s, K)
    AtA = np.zeros((kv.size, kv.size))
    V = d.u(s.ng * s.nz, -1, 1).reshape(s.ng, s.nz)
    adj = np.zeros(kv.size)
    for j in range(s.ng):
        Ah = linearize.A_hat_dense(s, j)
        assert np.allclose(Ah @ kv + s.bhat[j], E[j], atol=1e-13)
        AtA += Ah.T @ Ah
        adj += Ah.T @ V[j]
    assert np.allclose(AtA, linearize.AtA_dense(s), atol=1e-12)
    assert np.allclose(linearize.K_to_kv(linearize.eta_adjoint(s, V)), adj, atol=1e-12)
    # 1/2 k' Q_v k = sum_k ||R_K K_k||_F^2
    ref = sum(np.sum((prob.RK @ K[k]) ** 2) for k in range(s.T))
    assert 0.5 * kv @ linearize.Qv_dense(s) @ kv == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("make", [synth.config1, synth.config2, synth.config3])
def test_cone_support_is_compact(make):
    prob = make()
    prob.T = 5
    prob.u_init = prob.u_init[:5]
    s = linearize.assemble(prob, prob.u_init)
    T, nx, nu = s.T, s.nx, s.nu
    for j in range(s.ng):
        t = s.time[j]
        bh = s.bhat[j].reshape(T + 1, nx)
        b = s.bmat[j].reshape(T, nu)
        if s.kind[j] == linearize.KIND_STATE:
            assert np.all(bh[t + 1:] == 0.0) and np.all(b[t:] == 0.0)
        else:
            assert np.all(bh == 0.0)
            assert np.count_nonzero(b) == 1 and np.all(b[np.arange(T) != t] == 0.0)
