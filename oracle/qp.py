"""The (delta_u, p) block of both inner methods (the update written after the
DR subproblem in Section II-B and the first Block-2 update of Section IV):

    min_{du, p}  Q_u(du) + (rho/2) ||p - c||^2
    s.t.         g0 + B du + p <= 0,   ||F_u du||_2 <= r_trust

with c = p~ - lambda/rho (NRTO-DR) or c = p~ - lambda_p (FullADMM, scaled duals).

Solved exactly (the paper's preconditioned CG is replaced; see the design
notes): p is eliminated, p_j = min(c_j, -g0_j - b_j' du), leaving the convex
C^1 piecewise quadratic
    phi(du) = 1/2 du' H du + h' du + (rho/2) sum_j max(0, g0_j + b_j' du + c_j)^2,
minimised by semismooth Newton with an exact line search along each Newton
direction.  If the minimiser violates the trust region, the multiplier mu of
1/2 ||F_u du||^2 <= 1/2 r^2 is found by bisection on the non-increasing map
mu -> ||F_u du(mu)||.  Multipliers: pi_j = rho max(0, g0_j + b_j' du + c_j).
"""
from __future__ import annotations

import numpy as np


def _line_search(Hm, gvec, u, d, B, beta, rho):
    """Exact minimiser over s >= 0 of phi(u + s d) (piecewise quadratic in s)."""
    a = B @ u + beta
    e = B @ d
    dHd = float(d @ Hm @ d)
    g0 = float(d @ gvec)          # derivative of the smooth part at s = 0
    if dHd <= 0.0:
        return 0.0
    bps = []
    for j in range(len(a)):
        if e[j] != 0.0:
            s = -a[j] / e[j]
            if s > 0.0:
                bps.append(s)
    bps = sorted(set(bps))
    lo = 0.0
    for hi in bps + [np.inf]:
        mid = lo + 1.0 if hi == np.inf else 0.5 * (lo + hi)
        act = (a + mid * e) > 0.0
        # derivative on (lo, hi): slope * s + icpt
        slope = dHd + rho * float(e[act] @ e[act])
        icpt = g0 + rho * float(e[act] @ a[act])
        if slope > 0.0:
            s = -icpt / slope
            if s <= hi and s >= lo:
                return max(s, 0.0)
            if s < lo:
                return lo
        lo = hi
    return lo


def _ssn(Hm, h, B, beta, rho, u0, max_iter=100):
    """Semismooth Newton for min 1/2 u'Hm u + h'u + rho/2 sum max(0, Bu + beta)^2.

    Each step solves the Newton system of the current active set.  If the full
    step keeps that active set it is the exact minimiser and the loop ends;
    otherwise the exact line search picks the step length.
    """
    u = u0.copy()
    for _ in range(max_iter):
        a = B @ u + beta
        act = a > 0.0
        Ba = B[act]
        grad = Hm @ u + h + rho * Ba.T @ a[act]
        Hn = Hm + rho * Ba.T @ Ba
        d = -np.linalg.solve(Hn, grad)
        if not np.all(np.isfinite(d)):
            break
        full = u + d
        if np.array_equal((B @ full + beta) > 0.0, act):
            return full
        s = _line_search(Hm, Hm @ u + h, u, d, B, beta, rho)
        if s * np.max(np.abs(d)) <= 1e-15 * (1.0 + np.max(np.abs(u))):
            break
        u = u + s * d
    return u


def solve(H, h, B, g0, c, rho, Fu, r_trust, u_start=None):
    """Returns (du, p, pi, mu)."""
    n = H.shape[0]
    beta = g0 + c
    M = Fu.T @ Fu
    u0 = np.zeros(n) if u_start is None else u_start
    u = _ssn(H, h, B, beta, rho, u0)
    mu = 0.0
    psi = float(np.linalg.norm(Fu @ u))
    if psi > r_trust:
        lo, hi = 0.0, 1.0
        u_hi = _ssn(H + hi * M, h, B, beta, rho, u)
        while float(np.linalg.norm(Fu @ u_hi)) > r_trust:
            lo = hi
            hi *= 4.0
            u_hi = _ssn(H + hi * M, h, B, beta, rho, u_hi)
        um = u_hi
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            um = _ssn(H + mid * M, h, B, beta, rho, um)
            psi = float(np.linalg.norm(Fu @ um))
            if abs(psi - r_trust) <= 1e-13 * r_trust or (hi - lo) <= 1e-15 * hi:
                break
            if psi > r_trust:
                lo = mid
            else:
                hi = mid
        u, mu = um, mid
    a = B @ u + g0
    p = np.minimum(c, -a)
    pi = rho * np.maximum(0.0, a + c)
    return u, p, pi, mu


def objective(H, h, B, g0, c, rho, du, p):
    """Value of the subproblem objective 1/2 du'H du + h'du + rho/2 ||p - c||^2 (constant dropped)."""
    return float(0.5 * du @ H @ du + h @ du + 0.5 * rho * np.sum((p - c) ** 2))
