"""Pins of the oracle's learned-warm-start reconstruction (oracle/warm.py)
against what the DR splitting fixes (supplementary II-A): the rebuilt state is
a fixed point of the relaxed DR iteration wherever the prediction satisfies
complementarity and the gains need no change, the p~ prox and the cone
projection return the rebuilt point for any prediction, the KKT residual's
multiplier terms vanish at it, a converged solution of a problem whose optimal
gains are zero rebuilds to a point with the solve's residual, and the fallback
keeps the cold point for a bad prediction."""
import numpy as np

import synth
from oracle import dr, kkt, linearize, soc, warm
from oracle.linearize import eta


def _socp(radius=0.05, T=8):
    prob = synth.config1()
    prob.T = T
    prob.radius = radius
    prob.u_init = np.tile([1.0, 0.0], (T, 1))
    prob.obstacles = np.array([[0.45, 0.3, 0.15]])
    return linearize.assemble(prob, prob.u_init, 5.0)


def _opt(**kw):
    base = dict(rho=50.0, sigma_s=7.0, sigma_chi=1.0, alpha=1.0, cold_init="margin")
    base.update(kw)
    return dr.Options(**base)


def test_slack_prediction_is_a_dr_fixed_point():
    # pi = 0 and p~ above ||b_hat||: the rebuilt point is left unchanged by a DR step
    s = _socp()
    o = _opt()
    n = np.sqrt(np.sum(s.bhat ** 2, axis=1))
    pt_pred = n + 0.1 + synth.uniform(5, s.ng)
    du = 0.1 * (2 * synth.uniform(6, s.T * s.nu) - 1)
    st = warm.reconstruct(s, o, du, pt_pred, np.zeros(s.ng))
    s_t0, pt0 = st.s_t.copy(), st.pt.copy()
    dr.dr_steps(s, o, st, dr.factor(s, o), 1)
    assert np.max(np.abs(st.K)) == 0.0
    assert np.max(np.abs(st.pt - pt0)) <= 1e-14 * np.max(pt0)
    assert np.max(np.abs(st.s_t - s_t0)) <= 1e-14 * np.max(np.abs(s_t0))


def test_zero_radius_complementary_prediction_is_a_dr_fixed_point():
    # r = 0: b_hat = 0 and the optimal gains are zero; with pi_j > 0 only where
    # p~_j = 0 (complementarity) the rebuilt point is a DR fixed point
    s = _socp(radius=0.0)
    o = _opt()
    pi = np.where(synth.uniform(7, s.ng) < 0.5, 0.0, 1.0 + synth.uniform(8, s.ng))
    pt_pred = np.where(pi > 0, 0.0, synth.uniform(9, s.ng))
    st = warm.reconstruct(s, o, np.zeros(s.T * s.nu), pt_pred, pi)
    s_t0, pt0 = st.s_t.copy(), st.pt.copy()
    dr.dr_steps(s, o, st, dr.factor(s, o), 1)
    assert np.max(np.abs(st.K)) == 0.0
    assert np.max(np.abs(st.pt - pt0)) <= 1e-14
    assert np.max(np.abs(st.s_t - s_t0)) <= 1e-14 * max(1.0, np.max(np.abs(s_t0)))


def test_p_prox_and_projection_return_the_rebuilt_point():
    # any prediction: the p~ prox of the rebuilt state returns p~ exactly; a
    # complementary prediction (pi_j > 0 only where the rebuilt cone is active,
    # p~_j = ||eta_j||): the cone projection of the reflected affine point at
    # K = 0 returns that point
    s = _socp()
    o = _opt()
    pt_any = 2 * synth.uniform(10, s.ng) - 0.5
    pi_any = 3 * synth.uniform(11, s.ng) - 1.0
    st = warm.reconstruct(s, o, np.zeros(s.T * s.nu), pt_any, pi_any)
    pt_new = (o.sigma_chi * st.pt_t + o.rho * st.p + st.lam + o.sigma_s * st.s_t[:, 0]) / (o.rho + o.sigma_chi + o.sigma_s)
    assert np.max(np.abs(pt_new - st.pt)) <= 1e-13 * np.max(st.pt)
    n = np.sqrt(np.sum(s.bhat ** 2, axis=1))
    active = (synth.uniform(15, s.ng) < 0.5) & (n > 0)
    pi = np.where(active, 0.5 + synth.uniform(16, s.ng), 0.0)
    pt_pred = np.where(active, 0.5 * n, n + synth.uniform(17, s.ng))
    st = warm.reconstruct(s, o, np.zeros(s.T * s.nu), pt_pred, pi)
    S = np.concatenate([st.pt[:, None], eta(s, st.K)], axis=1)
    P = soc.project_rows_vec(2 * S - st.s_t)
    assert np.max(np.abs(P - S)) <= 1e-13 * np.max(np.abs(S))


def test_multiplier_terms_of_the_residual_vanish():
    s = _socp()
    o = _opt()
    st = warm.reconstruct(s, o, 0.05 * (2 * synth.uniform(12, s.T * s.nu) - 1),
                          synth.uniform(13, s.ng), 2 * synth.uniform(14, s.ng) - 0.5)
    t = kkt.terms(s, st.du, st.K, st.p, st.pt, st.pi, st.mu, dr.zeta(s, o, st))
    assert t[4] == 0.0                       # T5: p = p~
    assert t[6] <= 1e-15                     # T7: ||zeta_j|| <= pi_j
    assert t[7] <= 1e-14                     # T8: pi_j ||eta_j|| + zeta_j' eta_j = 0
    assert np.all(st.pt >= np.sqrt(np.sum(s.bhat ** 2, axis=1)))


def test_converged_zero_radius_solution_rebuilds_to_a_solution():
    s = _socp(radius=0.0)
    o = _opt(max_admm=400, max_dr=200, eps_kkt=1e-9, eps_dr_abs=1e-12, eps_dr_rel=1e-12, cold_init="zero")
    st, info = dr.solve(s, o)
    assert info["kkt"] <= 1e-9
    assert np.max(np.abs(st.K)) <= 1e-9
    w = warm.reconstruct(s, o, st.du, st.pt, st.pi)
    w.mu = st.mu
    assert dr.residual(s, o, w) <= 1e-8


def test_fallback_keeps_the_cold_point_for_a_bad_prediction():
    s = _socp()
    o = _opt()
    bad_du = 50.0 * np.ones(s.T * s.nu)
    st, keep, r_w, r_c = warm.warm_or_cold(s, o, bad_du, np.zeros(s.ng), 100.0 * np.ones(s.ng))
    assert not keep and r_w > r_c
    cold = dr.cold_state(s, o)
    assert np.array_equal(st.s_t, cold.s_t) and np.array_equal(st.du, cold.du)
