"""Pins of the oracle's cost data and quadrotor dynamics against definitions
computed by a different route.

* Q_u (the linearised nominal cost of Problem 2, with the tracking term the
  workloads add): the quadratic data (H, h, c0) must reproduce, for random du,
  the cost summed stage by stage over the deviations rolled forward with the
  per-step Jacobians (dx_{t+1} = A_t dx_t + B_t du_t, no F_u), and c0 must equal
  the nominal cost on the nonlinear rollout; the nonlinear cost of u + eps du
  must agree with Q_u(eps du) to second order in eps.
* Quadrotor (supplementary "Dynamical Models"): the thrust direction against
  the product of elementary rotations R = Rz(psi) Ry(theta) Rx(phi); the
  Euler-angle rate map against R'dR/dt = [omega]_x (body rates); Euler's
  rigid-body equations for the body rates; positions integrate velocities.
"""
import math

import numpy as np
import pytest

import synth
from oracle import linearize, models, scp


def _small(make, T):
    prob = make()
    prob.T = T
    prob.u_init = prob.u_init[:T]
    return prob


def _cost_by_stages(prob, s, du):
    """sum_k (u_k + du_k)' Ru (u_k + du_k) + sum_{t=1..T} (x_t + dx_t - xg)' Q (x_t + dx_t - xg)
    with dx rolled forward through the per-step Jacobians."""
    T, nx, nu = prob.T, prob.nx, prob.nu
    dU = du.reshape(T, nu)
    dx = np.zeros(nx)
    J = 0.0
    for k in range(T):
        uk = s.uhat[k] + dU[k]
        J += float(uk @ prob.Ru @ uk)
        dx = s.A[k] @ dx + s.B[k] @ dU[k]
        e = s.xhat[k + 1] + dx - prob.xg
        J += float(e @ prob.Q @ e)
    return J


@pytest.mark.parametrize("make,T", [(synth.config1, 7), (synth.config2, 6), (synth.config3, 5)])
def test_qu_data_equals_stagewise_cost(make, T):
    prob = _small(make, T)
    d = synth.Draws(17)
    u = prob.u_init + d.u(T * prob.nu, -0.2, 0.2).reshape(T, prob.nu)
    s = linearize.assemble(prob, u)
    # c0 is the nominal cost on the nonlinear rollout
    J0, _ = scp.nominal_cost(prob, u)
    assert abs(s.c0 - J0) <= 1e-12 * max(1.0, abs(J0))
    for _ in range(4):
        du = d.u(T * prob.nu, -1.0, 1.0)
        ref = _cost_by_stages(prob, s, du)
        assert abs(linearize.qu_value(s, du) - ref) <= 1e-12 * max(1.0, abs(ref))
    # the gradient at du = 0 and the Hessian, one column at a time, by the same stagewise sum
    n = T * prob.nu
    base = _cost_by_stages(prob, s, np.zeros(n))
    for i in range(0, n, max(1, n // 5)):
        e = np.zeros(n)
        e[i] = 1.0
        fp, fm = _cost_by_stages(prob, s, e), _cost_by_stages(prob, s, -e)
        # exact for a quadratic: h_i = (f(e) - f(-e)) / 2, H_ii = f(e) + f(-e) - 2 f(0)
        assert abs(s.h[i] - 0.5 * (fp - fm)) <= 1e-10 * max(1.0, abs(fp), abs(fm))
        assert abs(s.H[i, i] - (fp + fm - 2.0 * base)) <= 1e-10 * max(1.0, abs(fp), abs(fm))


@pytest.mark.parametrize("make,T", [(synth.config1, 7), (synth.config2, 6), (synth.config3, 5)])
def test_qu_is_second_order_model_of_nonlinear_cost(make, T):
    prob = _small(make, T)
    d = synth.Draws(23)
    u = prob.u_init + d.u(T * prob.nu, -0.2, 0.2).reshape(T, prob.nu)
    s = linearize.assemble(prob, u)
    du = d.u(T * prob.nu, -1.0, 1.0)
    errs = []
    for eps in (1e-2, 5e-3):
        J1, _ = scp.nominal_cost(prob, u + eps * du.reshape(T, prob.nu))
        errs.append(abs(J1 - linearize.qu_value(s, eps * du)))
    # first-order terms agree exactly, so halving eps cuts the error by about 4 (not 2)
    assert errs[1] <= 0.3 * errs[0] + 1e-13


def _rot(ph, th, ps):
    cx, sx, cy, sy, cz, sz = math.cos(ph), math.sin(ph), math.cos(th), math.sin(th), math.cos(ps), math.sin(ps)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def _quad():
    prob = synth.config2()
    prob.inertia = np.array([0.02, 0.025, 0.04])
    return prob


def test_quadrotor_level_thrust_and_yaw_rate():
    prob = _quad()
    for psi in (0.0, 0.7, -2.1):
        x = np.zeros(12)
        x[8] = psi
        x[9:12] = [0.0, 0.0, 0.3]
        f = 13.0
        xd = models.xdot(prob, x, np.array([f, 0.0, 0.0, 0.0]))
        # level attitude: thrust along world z, vdot_z = f/m - g, no horizontal force
        assert np.allclose(xd[3:6], [0.0, 0.0, f / prob.mass - models.G], atol=1e-14)
        # level attitude: psi_dot = r, phi_dot = p, theta_dot = q
        assert np.allclose(xd[6:9], [0.0, 0.0, 0.3], atol=1e-15)


def test_quadrotor_pure_body_torque():
    prob = _quad()
    x = np.zeros(12)
    tau = np.array([0.01, -0.02, 0.03])
    xd = models.xdot(prob, x, np.concatenate([[prob.mass * models.G], tau]))
    # at rest: p_dot = tau_x / J_x (and likewise), no translation
    assert np.allclose(xd[9:12], tau / prob.inertia, atol=1e-15)
    assert np.allclose(xd[3:6], 0.0, atol=1e-14)


def test_quadrotor_euler_rigid_body_equations():
    prob = _quad()
    J1, J2, J3 = prob.inertia
    d = synth.Draws(41)
    for _ in range(5):
        x = d.u(12, -0.5, 0.5)
        u = np.concatenate([[9.0], d.u(3, -0.05, 0.05)])
        p, q, r = x[9:12]
        xd = models.xdot(prob, x, u)
        ref = [(u[1] + (J2 - J3) * q * r) / J1, (u[2] + (J3 - J1) * r * p) / J2, (u[3] + (J1 - J2) * p * q) / J3]
        assert np.allclose(xd[9:12], ref, atol=1e-13)
        # positions integrate velocities
        assert np.array_equal(xd[0:3], x[3:6])


def test_quadrotor_thrust_direction_is_rotated_body_z():
    prob = _quad()
    d = synth.Draws(43)
    for _ in range(6):
        ph, th, ps = d.u(3, -1.2, 1.2)
        x = np.zeros(12)
        x[6:9] = [ph, th, ps]
        f = 7.5
        xd = models.xdot(prob, x, np.array([f, 0.0, 0.0, 0.0]))
        R = _rot(ph, th, ps)
        assert np.allclose(xd[3:6], (f / prob.mass) * R[:, 2] - np.array([0.0, 0.0, models.G]), atol=1e-13)


def test_quadrotor_euler_rates_match_body_rates():
    """The Euler-angle rates of xdot must make R(angles(t)) rotate with body rate
    omega: R' dR/dt = [omega]_x (checked by a central difference of R along the
    rates)."""
    prob = _quad()
    d = synth.Draws(47)
    for _ in range(6):
        ang = d.u(3, -1.0, 1.0)
        w = d.u(3, -2.0, 2.0)
        x = np.zeros(12)
        x[6:9] = ang
        x[9:12] = w
        rates = models.xdot(prob, x, np.array([9.81, 0.0, 0.0, 0.0]))[6:9]
        h = 1e-6
        dR = (_rot(*(ang + h * rates)) - _rot(*(ang - h * rates))) / (2 * h)
        W = _rot(*ang).T @ dR
        skew = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
        assert np.max(np.abs(W - skew)) <= 1e-7
