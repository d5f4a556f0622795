"""Pins of the oracle's NRTO-DR and NRTO-FullADMM:

* the reduced affine-set prox equals the solution of the full quasi-definite
  KKT system of supplementary II-B, solved densely;
* FullADMM keeps Q_v k_v + rho sum_j A_hat_j' lambda_nu_j = 0 (supplementary
  III) and its closed-form k_v step equals the standard ADMM k_v step;
* both methods reach the same unique (du*, k_v*) as an independent
  general-purpose NLP solver (SciPy SLSQP) on small problems;
* the ball radius r = 0 gives K* = 0 and the nominal QP solution.
"""
import numpy as np
import pytest
import scipy.optimize as so

import synth
from oracle import dr, fulladmm, kkt, linearize
from oracle.linearize import eta, eta_adjoint


def near_obstacle_socp(T=8, radius=0.05, r_trust=5.0):
    """Unicycle driving along x at 1 m/s past an obstacle just off its path,
    so the robust obstacle constraints are active and K* is nonzero."""
    prob = synth.config1()
    prob.T = T
    prob.radius = radius
    prob.u_init = np.tile([1.0, 0.0], (T, 1))
    prob.obstacles = np.array([[0.45, 0.3, 0.15]])
    return linearize.assemble(prob, prob.u_init, r_trust)


def dense_conic(s, rho, p, lam):
    """P, q, A, b of the DR standard form (supplementary II-A) written out."""
    n = s.T * s.nu * s.nx
    ng, nz = s.ng, s.nz
    P = np.zeros((n + ng, n + ng))
    P[:n, :n] = linearize.Qv_dense(s)
    P[n:, n:] = rho * np.eye(ng)
    q = np.concatenate([np.zeros(n), -(rho * p + lam)])
    A = np.zeros((ng * (1 + nz), n + ng))
    b = np.zeros(ng * (1 + nz))
    for j in range(ng):
        r0 = j * (1 + nz)
        A[r0, n + j] = -1.0
        A[r0 + 1:r0 + 1 + nz, :n] = -linearize.A_hat_dense(s, j)
        b[r0 + 1:r0 + 1 + nz] = s.bhat[j]
    return P, q, A, b


def test_reduced_prox_equals_full_kkt():
    s = near_obstacle_socp(T=3)
    o = dr.Options(rho=40.0, sigma_chi=0.7, sigma_s=1.3)
    d = synth.Draws(21)
    st = dr.zero_state(s)
    st.K_t = d.u(st.K_t.size, -1, 1).reshape(st.K_t.shape)
    st.pt_t = d.u(s.ng, -1, 1)
    st.s_t = d.u(st.s_t.size, -1, 1).reshape(st.s_t.shape)
    st.p = d.u(s.ng, -1, 1)
    st.lam = d.u(s.ng, -1, 1)
    chi_t = np.concatenate([linearize.K_to_kv(st.K_t), st.pt_t])
    s_t = st.s_t.ravel().copy()
    P, q, A, b = dense_conic(s, o.rho, st.p, st.lam)
    nchi, m = P.shape[0], A.shape[0]
    Kkkt = np.block([[P + o.sigma_chi * np.eye(nchi), A.T], [A, -np.eye(m) / o.sigma_s]])
    rhs = np.concatenate([o.sigma_chi * chi_t - q, b - s_t])
    sol = np.linalg.solve(Kkkt, rhs)
    chi, y = sol[:nchi], sol[nchi:]
    s_new = s_t - y / o.sigma_s
    assert np.max(np.abs(Kkkt @ sol - rhs)) <= 1e-12
    # one oracle DR step records chi = (K, p~) of its prox
    dr.dr_steps(s, o, st, dr.factor(s, o), 1)
    n = s.T * s.nu * s.nx
    assert np.allclose(linearize.K_to_kv(st.K), chi[:n], atol=1e-12)
    assert np.allclose(st.pt, chi[n:], atol=1e-12)
    S = np.concatenate([st.pt[:, None], eta(s, st.K)], axis=1).ravel()
    assert np.allclose(S, s_new, atol=1e-12)


def test_fulladmm_invariant_and_standard_step():
    s = near_obstacle_socp()
    o = fulladmm.Options(rho=10.0, max_admm=1)
    st = fulladmm.zero_state(s)
    fac = fulladmm.factor(s, o)
    for _ in range(25):
        K_prev, lam_prev = st.K.copy(), st.lam_nu.copy()
        fulladmm.iterate(s, o, st, fac)
        inv = fulladmm.invariant(s, o, st)
        assert np.max(np.abs(inv)) <= 1e-12 * (1 + np.max(np.abs(st.K)) + o.rho * np.max(np.abs(st.lam_nu)))
        # standard step: (Q_v + rho sum A'A) k = -rho sum A'(b_hat - nu + lambda_nu_prev)
        n = s.T * s.nu * s.nx
        M = linearize.Qv_dense(s) + o.rho * linearize.AtA_dense(s)
        rhs = -o.rho * linearize.K_to_kv(eta_adjoint(s, s.bhat - st.nu_ + lam_prev))
        assert np.allclose(np.linalg.solve(M, rhs), linearize.K_to_kv(st.K), atol=1e-10)


def _slsqp(s):
    """Problem 2 with p eliminated, solved by SLSQP in (du, k_v)."""
    nd = s.T * s.nu
    nk = s.T * s.nu * s.nx
    Qv = linearize.Qv_dense(s)

    def f(z):
        du, kv = z[:nd], z[nd:]
        return 0.5 * du @ s.H @ du + s.h @ du + 0.5 * kv @ Qv @ kv

    def cons(z):
        du, kv = z[:nd], z[nd:]
        E = eta(s, linearize.kv_to_K(kv, s.T, s.nu, s.nx))
        return -(s.g0 + s.bmat @ du + np.sqrt(np.sum(E * E, axis=1) + 1e-30))

    def trust(z):
        return s.r_trust ** 2 - np.sum((s.Fu @ z[:nd]) ** 2)

    z0 = np.zeros(nd + nk)
    res = so.minimize(f, z0, method="SLSQP", constraints=[{"type": "ineq", "fun": cons},
                                                          {"type": "ineq", "fun": trust}],
                      options={"ftol": 1e-14, "maxiter": 2000})
    return res.x[:nd], linearize.kv_to_K(res.x[nd:], s.T, s.nu, s.nx)


def test_methods_agree_with_independent_solver():
    s = near_obstacle_socp(T=6)
    od = dr.Options(max_dr=1000, max_admm=300, eps_kkt=1e-7, eps_dr_abs=1e-9, eps_dr_rel=1e-9)
    sd, idr = dr.solve(s, od)
    of = fulladmm.Options(max_admm=20000, eps_kkt=1e-8)
    sf, ifa = fulladmm.solve(s, of)
    assert idr["kkt"] <= 1e-7 and ifa["kkt"] <= 1e-8
    assert np.max(np.abs(sd.K)) > 1e-3          # the gains matter on this problem
    du_ref, K_ref = _slsqp(s)
    assert np.allclose(sd.du, sf.du, atol=2e-5)
    assert np.allclose(sd.K, sf.K, atol=2e-5)
    assert np.allclose(sd.du, du_ref, atol=2e-5)
    assert np.allclose(sd.K, K_ref, atol=2e-5)


def test_zero_radius_gives_zero_gain_and_nominal_qp():
    s = near_obstacle_socp(T=6, radius=0.0)
    sd, info = fulladmm.solve(s, fulladmm.Options(max_admm=20000, eps_kkt=1e-10))
    assert np.max(np.abs(sd.K)) <= 1e-12
    nd = s.T * s.nu
    res = so.minimize(lambda u: 0.5 * u @ s.H @ u + s.h @ u, np.zeros(nd), method="SLSQP",
                      constraints=[{"type": "ineq", "fun": lambda u: -(s.g0 + s.bmat @ u)},
                                   {"type": "ineq", "fun": lambda u: s.r_trust ** 2 - np.sum((s.Fu @ u) ** 2)}],
                      options={"ftol": 1e-15, "maxiter": 1000})
    assert np.allclose(sd.du, res.x, atol=1e-6)


def test_dr_fixed_point_certificate():
    # at convergence y_hat = sigma_s (s_hat - s_ref) is in K and orthogonal to s_hat
    s = near_obstacle_socp(T=5)
    o = dr.Options(max_dr=4000, max_admm=1, eps_dr_abs=1e-12, eps_dr_rel=1e-12, eps_kkt=0)
    st, _ = dr.solve(s, o)
    S = np.concatenate([st.pt[:, None], eta(s, st.K)], axis=1)
    S_ref = 2 * S - st.s_t
    from oracle.soc import project_rows_vec
    S_hat = project_rows_vec(S_ref)
    Y = o.sigma_s * (S_hat - S_ref)
    assert np.all(np.linalg.norm(Y[:, 1:], axis=1) <= Y[:, 0] + 1e-9)
    assert np.max(np.abs(np.sum(Y * S_hat, axis=1))) <= 1e-9
    assert np.max(np.abs(S_hat - S)) <= 1e-9


def _trust_region_minimiser(s):
    """min 1/2 du'H du + h'du s.t. ||F_u du|| <= r_trust through the secular
    equation: du(mu) = -(H + mu F'F)^-1 h, mu = 0 if it is inside, else the root
    of ||F_u du(mu)|| = r_trust (Brent)."""
    FtF = s.Fu.T @ s.Fu

    def du(mu):
        return np.linalg.solve(s.H + mu * FtF, -s.h)

    if np.linalg.norm(s.Fu @ du(0.0)) <= s.r_trust:
        return du(0.0), 0.0
    hi = 1.0
    while np.linalg.norm(s.Fu @ du(hi)) > s.r_trust:
        hi *= 4.0
    mu = so.brentq(lambda m: np.linalg.norm(s.Fu @ du(m)) - s.r_trust, 0.0, hi, xtol=1e-14, rtol=1e-14)
    return du(mu), mu


def slack_quadrotor_socp():
    """Hovering quadrotor far from its obstacles: every robust cone is slack at
    k_v = 0, so Problem 2's solution is K* = 0 and du* = the trust-region
    minimiser of Q_u (the trust region is active)."""
    prob = synth.config2()
    prob.T = 12
    prob.u_init = prob.u_init[:12]
    s = linearize.assemble(prob, prob.u_init, 0.5)
    assert np.max(s.g0 + np.linalg.norm(s.bhat, axis=1)) < 0
    return s


def test_margin_cold_point_solves_slack_problem_in_one_step():
    s = slack_quadrotor_socp()
    du_ref, mu_ref = _trust_region_minimiser(s)
    assert mu_ref > 0
    st, info = dr.solve(s, dr.Options(cold_init="margin", max_admm=5, eps_kkt=1e-9))
    assert info["admm_iters"] == 1 and info["dr_iters"] == 1
    assert np.max(np.abs(st.K)) == 0.0 and np.max(st.pi) == 0.0
    assert np.allclose(st.du, du_ref, rtol=1e-8, atol=1e-10)
    assert abs(st.mu - mu_ref) <= 1e-7 * mu_ref
    # from the printed zero point the same problem is not solved in 5 iterations
    _, info0 = dr.solve(s, dr.Options(max_admm=5, eps_kkt=1e-9))
    assert info0["kkt"] > 1e-6


def test_margin_cold_point_keeps_the_solution():
    s = near_obstacle_socp(T=5)
    o = dict(rho=200.0, sigma_s=10.0, max_dr=1000, max_admm=400, eps_kkt=1e-7, eps_dr_abs=1e-9, eps_dr_rel=1e-9)
    s0, i0 = dr.solve(s, dr.Options(**o))
    s1, i1 = dr.solve(s, dr.Options(cold_init="margin", **o))
    assert i0["kkt"] <= 1e-7 and i1["kkt"] <= 1e-7
    assert np.max(np.abs(s0.K)) > 1e-3
    assert np.allclose(s0.du, s1.du, atol=2e-5) and np.allclose(s0.K, s1.K, atol=2e-5)


def test_residual_balancing_keeps_the_solution_and_bounds():
    s = near_obstacle_socp(T=5)
    o = dict(rho=200.0, sigma_s=10.0, max_dr=1000, max_admm=600, eps_kkt=1e-7, eps_dr_abs=1e-9, eps_dr_rel=1e-9)
    s0, i0 = dr.solve(s, dr.Options(**o))
    s1, i1 = dr.solve(s, dr.Options(rho_adapt=True, rho_min=5.0, rho_max=800.0, **o))
    assert i0["kkt"] <= 1e-7 and i1["kkt"] <= 1e-7
    assert i1["rho"] != 200.0 and 5.0 <= i1["rho"] <= 800.0
    assert np.allclose(s0.du, s1.du, atol=2e-5) and np.allclose(s0.K, s1.K, atol=2e-5)
    # the penalty only moves by the factor tau inside [rho_min, rho_max]
    lg = np.log2(i1["rho"] / 200.0)
    assert abs(lg - round(lg)) < 1e-12


def test_sigma_balancing_keeps_the_solution():
    s = near_obstacle_socp(T=5)
    o = dict(rho=200.0, sigma_s=10.0, max_dr=1000, max_admm=400, eps_kkt=1e-7, eps_dr_abs=1e-9, eps_dr_rel=1e-9)
    s0, i0 = dr.solve(s, dr.Options(**o))
    s1, i1 = dr.solve(s, dr.Options(sigma_adapt=True, sigma_every=5, sigma_thr=1.5, **o))
    assert i0["kkt"] <= 1e-7 and i1["kkt"] <= 1e-7
    assert i1["sigma_s"] != 10.0
    assert np.allclose(s0.du, s1.du, atol=2e-5) and np.allclose(s0.K, s1.K, atol=2e-5)
    # the returned multipliers are consistent with the final scaling
    z = dr.zeta(s, dr.Options(**o), s1)
    assert np.allclose(z, s1.sigma_s * (s1.s_t[:, 1:] - eta(s, s1.K)))


def test_sigma_rescale_keeps_a_fixed_point():
    # at a DR fixed point S = S_hat, so the rescale s~ <- S + f (s~ - S) with the
    # refactored scaling leaves (K, p~) fixed: one more DR step moves nothing
    s = near_obstacle_socp(T=5)
    o = dr.Options(rho=200.0, sigma_s=10.0, eps_dr_abs=1e-13, eps_dr_rel=1e-13, cold_init="margin")
    st = dr.cold_state(s, o)
    st.p[:] = 0.3
    st.lam[:] = 1.0
    n, r_dr, _ = dr.dr_steps(s, o, st, dr.factor(s, o), 6000)
    assert r_dr <= 1e-11
    S = np.concatenate([st.pt[:, None], eta(s, st.K)], axis=1)
    f = 0.25
    st.s_t = S + f * (st.s_t - S)
    st.sigma_s = o.sigma_s / f
    K0, pt0 = st.K.copy(), st.pt.copy()
    dr.dr_steps(s, o, st, dr.factor(s, o, st.sigma_s), 1)
    assert np.max(np.abs(st.K - K0)) <= 1e-8 and np.max(np.abs(st.pt - pt0)) <= 1e-8
