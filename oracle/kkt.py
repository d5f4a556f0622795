"""One FP64 KKT residual of the tractable linearised problem (Problem 2).

The paper stops its inner loops on fixed-point and ADMM residuals and never
defines a solution accuracy; this residual (a reading) is what "solved to
1e-4" means here.  Problem 2 in conic form has multipliers
  pi_j >= 0           for  g0_j + b_j' du + p_j <= 0,
  (pi_j, zeta_j) in K for  (p_j, eta_j) in K_j (p-stationarity makes the
                           cone's scalar multiplier equal pi_j; K is self-dual),
  mu >= 0             for  1/2 ||F_u du||^2 <= 1/2 r_trust^2,
so the stationarity conditions are
  grad Q_u(du) + B' pi + mu F_u'F_u du = 0,   Q_v k_v - sum_j A_hat_j' zeta_j = 0.
The inner methods supply zeta: NRTO-DR  zeta_j = sigma_s (eta~_j - eta_j) (the
multiplier y of the affine-set prox, eta~ from the DR state); FullADMM
zeta_j = -rho lambda_nu_j.  With e_j = g0_j + b_j' du, eta_j = A_hat_j k_v + b_hat_j,
n_j = ||eta_j||:

  T1  ||grad Q_u + B' pi + mu F_u'F_u du||_inf / (1 + max of the three norms)
  T2  ||Q_v k_v - sum_j A_hat_j' zeta_j||_inf / (1 + max of the two norms)
  T3  max_j (e_j + n_j)_+ / (1 + max_j max(|g0_j|, |b_j' du|, n_j))
  T4  (||F_u du|| - r_trust)_+ / (1 + r_trust)
  T5  ||p - p~||_inf / (1 + max(||p||_inf, ||p~||_inf))
  T6  max_j |min(pi_j, -(e_j + n_j))| / (1 + max_j max(pi_j, |e_j|, n_j))
  T7  max_j max((-pi_j)_+, (||zeta_j|| - pi_j)_+) / (1 + ||pi||_inf)
  T8  max_j |pi_j n_j + zeta_j' eta_j| / (1 + max_j pi_j n_j)
  T9  |min(mu, r_trust - ||F_u du||)| / (1 + max(mu, r_trust))

residual = max(T1..T9).
"""
from __future__ import annotations

import numpy as np

from .linearize import eta, eta_adjoint


def terms(socp, du, K, p, pt, pi, mu, zeta):
    bdu = socp.bmat @ du
    e = socp.g0 + bdu
    E = eta(socp, K)
    n = np.sqrt(np.sum(E * E, axis=1))
    gq = socp.H @ du + socp.h
    bpi = socp.bmat.T @ pi
    Fdu = socp.Fu @ du
    tr = mu * (socp.Fu.T @ Fdu)
    t1 = np.max(np.abs(gq + bpi + tr)) / (1.0 + max(np.max(np.abs(gq)), np.max(np.abs(bpi)), np.max(np.abs(tr))))
    qk = 2.0 * np.einsum("uv,kvx->kux", socp.RK2, K)
    az = eta_adjoint(socp, zeta)
    t2 = np.max(np.abs(qk - az)) / (1.0 + max(np.max(np.abs(qk)), np.max(np.abs(az))))
    viol = e + n
    t3 = max(0.0, np.max(viol)) / (1.0 + max(np.max(np.abs(socp.g0)), np.max(np.abs(bdu)), np.max(n)))
    nf = float(np.linalg.norm(Fdu))
    t4 = max(0.0, nf - socp.r_trust) / (1.0 + socp.r_trust)
    t5 = np.max(np.abs(p - pt)) / (1.0 + max(np.max(np.abs(p)), np.max(np.abs(pt))))
    t6 = np.max(np.abs(np.minimum(pi, -viol))) / (1.0 + max(np.max(pi), np.max(np.abs(e)), np.max(n)))
    zn = np.sqrt(np.sum(zeta * zeta, axis=1))
    t7 = max(0.0, np.max(np.maximum(-pi, zn - pi))) / (1.0 + np.max(np.abs(pi)))
    t8 = np.max(np.abs(pi * n + np.sum(zeta * E, axis=1))) / (1.0 + np.max(pi * n))
    t9 = abs(min(mu, socp.r_trust - nf)) / (1.0 + max(mu, socp.r_trust))
    return np.array([t1, t2, t3, t4, t5, t6, t7, t8, t9])


def residual(socp, du, K, p, pt, pi, mu, zeta) -> float:
    return float(np.max(terms(socp, du, K, p, pt, pi, mu, zeta)))
