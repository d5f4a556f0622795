"""Dynamics and analytic Jacobians (supplementary material, "Dynamical Models").

All three models are discretised with forward Euler, x_{k+1} = x_k + dt * xdot.
Input saturation and state clipping from the paper's simulators are not part
of the optimisation model: bounds enter as robust constraints instead.

  unicycle  x = (px, py, theta), u = (v, omega)
  quadrotor x = (p, v, phi, theta, psi, omega), u = (f, tau); R = Rz Ry Rx,
            body-z thrust, Euler-angle rate map T(phi, theta), J diagonal
  arm       x = (q, qdot) in R^14, u = qddot in R^7 (joint-space double
            integrator); obstacle distances use a 7-link standard-DH chain
"""
from __future__ import annotations

import math

import numpy as np

G = 9.81


def _alpha_dh(i: int) -> float:
    """DH twist of link i (0-based): +pi/2 for odd links (1-based), -pi/2 for even, 0 for the last."""
    if i == 6:
        return 0.0
    return math.pi / 2 if i % 2 == 0 else -math.pi / 2


def xdot(prob, x: np.ndarray, u: np.ndarray) -> np.ndarray:
    if prob.dyn == 0:
        return np.array([u[0] * math.cos(x[2]), u[0] * math.sin(x[2]), u[1]])
    if prob.dyn == 1:
        m = prob.mass
        J = prob.inertia
        ph, th, ps = x[6], x[7], x[8]
        w = x[9:12]
        cph, sph, cth, sth, cps, sps = math.cos(ph), math.sin(ph), math.cos(th), math.sin(th), math.cos(ps), math.sin(ps)
        Re3 = np.array([cps * sth * cph + sps * sph, sps * sth * cph - cps * sph, cth * cph])
        vdot = np.array([0.0, 0.0, -G]) + (u[0] / m) * Re3
        Tm = np.array([[1.0, sph * math.tan(th), cph * math.tan(th)],
                       [0.0, cph, -sph],
                       [0.0, sph / cth, cph / cth]])
        angdot = Tm @ w
        Jw = J * w
        wdot = (u[1:4] - np.cross(w, Jw)) / J
        return np.concatenate([x[3:6], vdot, angdot, wdot])
    if prob.dyn == 2:
        return np.concatenate([x[7:14], u])
    raise ValueError("unknown dynamics")


def step(prob, x: np.ndarray, u: np.ndarray) -> np.ndarray:
    """One forward-Euler step x + dt * xdot(x, u)."""
    return x + prob.dt * xdot(prob, x, u)


def jacobians(prob, x: np.ndarray, u: np.ndarray):
    """Analytic A = d step / dx and B = d step / du."""
    nx, nu, dt = prob.nx, prob.nu, prob.dt
    Fx = np.zeros((nx, nx))
    Fu = np.zeros((nx, nu))
    if prob.dyn == 0:
        th = x[2]
        Fx[0, 2] = -u[0] * math.sin(th)
        Fx[1, 2] = u[0] * math.cos(th)
        Fu[0, 0] = math.cos(th)
        Fu[1, 0] = math.sin(th)
        Fu[2, 1] = 1.0
    elif prob.dyn == 1:
        m = prob.mass
        J = prob.inertia
        ph, th, ps = x[6], x[7], x[8]
        p_, q_, r_ = x[9], x[10], x[11]
        cph, sph, cth, sth, cps, sps = math.cos(ph), math.sin(ph), math.cos(th), math.sin(th), math.cos(ps), math.sin(ps)
        tth = math.tan(th)
        f = u[0]
        # position rates
        Fx[0:3, 3:6] = np.eye(3)
        # thrust direction R e3 and its angle derivatives
        Re3 = np.array([cps * sth * cph + sps * sph, sps * sth * cph - cps * sph, cth * cph])
        dR_dph = np.array([-cps * sth * sph + sps * cph, -sps * sth * sph - cps * cph, -cth * sph])
        dR_dth = np.array([cps * cth * cph, sps * cth * cph, -sth * cph])
        dR_dps = np.array([-sps * sth * cph + cps * sph, cps * sth * cph + sps * sph, 0.0])
        Fx[3:6, 6] = (f / m) * dR_dph
        Fx[3:6, 7] = (f / m) * dR_dth
        Fx[3:6, 8] = (f / m) * dR_dps
        Fu[3:6, 0] = Re3 / m
        # Euler angle rates
        sec2 = 1.0 / (cth * cth)
        Fx[6, 6] = cph * tth * q_ - sph * tth * r_
        Fx[6, 7] = sph * sec2 * q_ + cph * sec2 * r_
        Fx[7, 6] = -sph * q_ - cph * r_
        Fx[8, 6] = (cph * q_ - sph * r_) / cth
        Fx[8, 7] = (sph * q_ + cph * r_) * sth / (cth * cth)
        Fx[6:9, 9:12] = np.array([[1.0, sph * tth, cph * tth],
                                  [0.0, cph, -sph],
                                  [0.0, sph / cth, cph / cth]])
        # body rates: wdot = J^-1 (tau - w x J w), J diagonal
        J1, J2, J3 = J
        Fx[9, 10] = -(J3 - J2) * r_ / J1
        Fx[9, 11] = -(J3 - J2) * q_ / J1
        Fx[10, 9] = -(J1 - J3) * r_ / J2
        Fx[10, 11] = -(J1 - J3) * p_ / J2
        Fx[11, 9] = -(J2 - J1) * q_ / J3
        Fx[11, 10] = -(J2 - J1) * p_ / J3
        Fu[9, 1] = 1.0 / J1
        Fu[10, 2] = 1.0 / J2
        Fu[11, 3] = 1.0 / J3
    elif prob.dyn == 2:
        Fx[0:7, 7:14] = np.eye(7)
        Fu[7:14, :] = np.eye(7)
    else:
        raise ValueError("unknown dynamics")
    return np.eye(nx) + dt * Fx, dt * Fu


def dh_frames(links: np.ndarray, q: np.ndarray):
    """Origins o_0..o_7 and z-axes z_0..z_7 of the standard-DH chain
    (a_i = L_i, d_i = 0, theta_i = q_i, alpha as in `_alpha_dh`)."""
    Tm = np.eye(4)
    origins = [Tm[:3, 3].copy()]
    zaxes = [Tm[:3, 2].copy()]
    for i in range(7):
        al = _alpha_dh(i)
        ct, st = math.cos(q[i]), math.sin(q[i])
        ca, sa = math.cos(al), math.sin(al)
        Ai = np.array([[ct, -st * ca, st * sa, links[i] * ct],
                       [st, ct * ca, -ct * sa, links[i] * st],
                       [0.0, sa, ca, 0.0],
                       [0.0, 0.0, 0.0, 1.0]])
        Tm = Tm @ Ai
        origins.append(Tm[:3, 3].copy())
        zaxes.append(Tm[:3, 2].copy())
    return np.array(origins), np.array(zaxes)


def link_points(links, q):
    """The 7 tested points: origins of DH frames 1..7."""
    o, _ = dh_frames(links, q)
    return o[1:]


def link_point_jacobian(links, q, i: int) -> np.ndarray:
    """3x7 Jacobian of link point i (0-based, frame i+1) w.r.t. q: revolute joint m
    moves it by z_{m} x (o_{i+1} - o_{m}) for m <= i."""
    o, z = dh_frames(links, q)
    Jp = np.zeros((3, 7))
    for mj in range(i + 1):
        Jp[:, mj] = np.cross(z[mj], o[i + 1] - o[mj])
    return Jp
