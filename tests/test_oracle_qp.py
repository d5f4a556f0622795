"""Pins of the exact (du, p) subproblem solver: brute-force enumeration of all
active sets on small instances, the subproblem's KKT conditions, the
trust-region multiplier, and the elimination of p."""
import itertools

import numpy as np
import pytest

import synth
from oracle import qp


def _rand_qp(seed, n, m):
    d = synth.Draws(seed)
    L = d.u(n * n, -1, 1).reshape(n, n)
    H = L @ L.T + 0.5 * np.eye(n)
    h = d.u(n, -2, 2)
    B = d.u(m * n, -1, 1).reshape(m, n)
    g0 = d.u(m, -1.0, 0.5)
    c = d.u(m, -0.5, 0.5)
    Fu = d.u(2 * n * n, -1, 1).reshape(2 * n, n)
    return H, h, B, g0, c, Fu


def _brute(H, h, B, beta, rho):
    """min over all active sets S of the quadratic with rows S active, keeping the
    candidate whose own active set is S (the piecewise-quadratic minimiser)."""
    m = B.shape[0]
    best = None
    for r in range(m + 1):
        for S in itertools.combinations(range(m), r):
            S = list(S)
            Bs = B[S]
            u = -np.linalg.solve(H + rho * Bs.T @ Bs, h + rho * Bs.T @ beta[S])
            act = set(np.nonzero(B @ u + beta > 0)[0].tolist())
            if act == set(S):
                val = 0.5 * u @ H @ u + h @ u + 0.5 * rho * np.sum(np.maximum(0, B @ u + beta) ** 2)
                if best is None or val < best[0]:
                    best = (val, u)
    return best[1]


@pytest.mark.parametrize("seed", range(6))
def test_matches_active_set_enumeration(seed):
    H, h, B, g0, c, Fu = _rand_qp(seed, 5, 8)
    rho = 10.0
    du, p, pi, mu = qp.solve(H, h, B, g0, c, rho, Fu, 1e9)
    assert mu == 0.0
    ref = _brute(H, h, B, g0 + c, rho)
    assert np.allclose(du, ref, atol=1e-11)
    # p eliminated exactly, multiplier from the squared hinge
    assert np.allclose(p, np.minimum(c, -(g0 + B @ du)))
    assert np.allclose(pi, rho * np.maximum(0, g0 + B @ du + c))


@pytest.mark.parametrize("seed", range(6))
def test_kkt_of_subproblem_with_trust_region(seed):
    H, h, B, g0, c, Fu = _rand_qp(100 + seed, 6, 10)
    rho = 7.0
    du0, *_ = qp.solve(H, h, B, g0, c, rho, Fu, 1e9)
    r = 0.3 * np.linalg.norm(Fu @ du0)
    du, p, pi, mu = qp.solve(H, h, B, g0, c, rho, Fu, r)
    assert mu > 0
    assert np.linalg.norm(Fu @ du) == pytest.approx(r, rel=1e-12)
    # stationarity in du of  Q(du) + rho/2||p - c||^2 with multipliers pi (linear) and mu
    g = H @ du + h + B.T @ pi + mu * Fu.T @ (Fu @ du)
    assert np.max(np.abs(g)) <= 1e-9 * (1 + np.max(np.abs(h)))
    # stationarity in p: rho (p - c) + pi = 0; feasibility; complementarity
    assert np.allclose(rho * (p - c) + pi, 0.0, atol=1e-12)
    assert np.all(g0 + B @ du + p <= 1e-12)
    assert np.all(pi >= 0) and np.max(np.abs(pi * (g0 + B @ du + p))) <= 1e-10
    # a smaller radius cannot give a lower-objective feasible point: compare with
    # random feasible perturbations along the sphere
    f = lambda u: 0.5 * u @ H @ u + h @ u + 0.5 * rho * np.sum(np.maximum(0, B @ u + g0 + c) ** 2)
    d = synth.Draws(seed + 500)
    for _ in range(50):
        v = du + 0.05 * d.u(du.size, -1, 1)
        nv = np.linalg.norm(Fu @ v)
        if nv > r:
            v = v * (r / nv)
        assert f(v) >= f(du) - 1e-10
