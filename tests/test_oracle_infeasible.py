"""The oracle's stop rule for infeasible linearisations (NRTO-DR option
infeas_window): an obstacle the nominal trajectory passes through cannot be
cleared inside a tiny trust region, so the linearised SOCP is infeasible and
the consensus residual ||p - p~|| stalls at a positive value; the same problem
with a large trust region is feasible and solves without the rule firing.
The KKT check schedule includes the last ADMM iteration."""
import numpy as np

import synth
from oracle import dr, linearize


def blocked_problem(T=8):
    prob = synth.config1()
    prob.T = T
    prob.radius = 0.02
    prob.u_init = np.tile([1.0, 0.0], (T, 1))
    prob.obstacles = np.array([[0.5, 0.04, 0.06]])   # crossed by the nominal path
    return prob


def _opt(**kw):
    base = dict(rho=50.0, sigma_s=10.0, cold_init="margin", max_admm=300, max_dr=100, eps_kkt=1e-4,
                infeas_window=20)
    base.update(kw)
    return dr.Options(**base)


def test_tiny_trust_region_is_reported_infeasible():
    prob = blocked_problem()
    s = linearize.assemble(prob, prob.u_init, 1e-3)
    assert np.max(s.g0) > 0.01                       # the nominal violates the obstacle
    st, info = dr.solve(s, _opt())
    assert info["status"] == "infeasible"
    assert info["admm_iters"] < 300
    assert info["r_p"] > 1e-3 * (1 + np.linalg.norm(st.pt))


def test_large_trust_region_solves_without_the_rule_firing():
    prob = blocked_problem()
    s = linearize.assemble(prob, prob.u_init, 5.0)
    st, info = dr.solve(s, _opt())
    assert info["status"] == "ok" and info["kkt"] <= 1e-4


def test_check_at_the_last_iteration():
    prob = blocked_problem()
    s = linearize.assemble(prob, prob.u_init, 5.0)
    _, ref = dr.solve(s, _opt(infeas_window=0))
    n = ref["admm_iters"]
    assert n >= 3
    # a schedule that never lands on the converged iteration except as the last one
    _, info = dr.solve(s, _opt(infeas_window=0, check_every=10 * n, max_admm=n))
    assert info["status"] == "ok" and info["admm_iters"] == n
