"""Pins of the oracle's dynamics Jacobians and arm kinematics: central finite
differences (h = 1e-6) of the forward-Euler steps, and closed forms of the
kinematics (a fully stretched chain, the base-joint rotation)."""
import math

import numpy as np
import pytest

import synth
from oracle import models


def _fd_jac(prob, x, u, h=1e-6):
    nx, nu = prob.nx, prob.nu
    A = np.zeros((nx, nx))
    B = np.zeros((nx, nu))
    for i in range(nx):
        e = np.zeros(nx)
        e[i] = h
        A[:, i] = (models.step(prob, x + e, u) - models.step(prob, x - e, u)) / (2 * h)
    for i in range(nu):
        e = np.zeros(nu)
        e[i] = h
        B[:, i] = (models.step(prob, x, u + e) - models.step(prob, x, u - e)) / (2 * h)
    return A, B


@pytest.mark.parametrize("make", [synth.config1, synth.config2, synth.config3])
def test_jacobians_match_finite_differences(make):
    prob = make()
    if prob.dyn == 1:
        prob.inertia = np.array([0.02, 0.025, 0.04])     # exercise the gyroscopic terms
    d = synth.Draws(99)
    for _ in range(5):
        x = d.u(prob.nx, -1.0, 1.0)
        u = d.u(prob.nu, -1.0, 1.0)
        A, B = models.jacobians(prob, x, u)
        Af, Bf = _fd_jac(prob, x, u)
        assert np.max(np.abs(A - Af)) <= 1e-7 * (1 + np.max(np.abs(A)))
        assert np.max(np.abs(B - Bf)) <= 1e-7 * (1 + np.max(np.abs(B)))


def test_quadrotor_hover_is_equilibrium():
    prob = synth.config2()
    x = np.zeros(12)
    u = np.array([prob.mass * models.G, 0, 0, 0])
    assert np.max(np.abs(models.step(prob, x, u) - x)) <= 1e-15


def test_unicycle_closed_form_step():
    prob = synth.config1()
    x = np.array([1.0, 2.0, 0.3])
    u = np.array([1.5, -0.7])
    ref = x + 0.1 * np.array([1.5 * math.cos(0.3), 1.5 * math.sin(0.3), -0.7])
    assert np.allclose(models.step(prob, x, u), ref, atol=1e-15)


def test_arm_kinematics_stretched_and_jacobian():
    prob = synth.config3()
    L = prob.links
    # q = 0: alternating +-pi/2 twists keep every a_i along the base x axis
    pts = models.link_points(L, np.zeros(7))
    assert np.allclose(pts[-1], [L.sum(), 0.0, 0.0], atol=1e-14)
    # rotating joint 1 by phi rotates the whole chain about the base z axis
    phi = 0.7
    q = np.zeros(7)
    q[0] = phi
    p = models.link_points(L, q)[-1]
    assert np.allclose(p, [L.sum() * math.cos(phi), L.sum() * math.sin(phi), 0.0], atol=1e-14)
    d = synth.Draws(5)
    for _ in range(3):
        q = d.u(7, -1.5, 1.5)
        for i in range(7):
            J = models.link_point_jacobian(L, q, i)
            Jf = np.zeros((3, 7))
            for m in range(7):
                e = np.zeros(7)
                e[m] = 1e-6
                Jf[:, m] = (models.link_points(L, q + e)[i] - models.link_points(L, q - e)[i]) / 2e-6
            assert np.max(np.abs(J - Jf)) <= 1e-8
