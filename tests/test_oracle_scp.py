"""The successive-linearisation step of the oracle (trust-region reading of the
outer-loop hyperparameter tables): a step is taken only when its SOCP was
solved to the KKT tolerance, and the radius then grows or stays; a step whose
solve stopped at the iteration cap is rejected and the radius shrinks by 0.8."""
import numpy as np

import synth
from oracle import dr, scp


def test_unsolved_step_is_rejected_and_radius_shrinks():
    prob = synth.config1()
    o = dr.Options(max_admm=1, max_dr=5, eps_kkt=1e-4)
    res = scp.step(prob, prob.u_init, 2.0, "dr", o)
    assert res.info["status"] == "maxiter"
    assert res.kkt > 1e-4
    assert not res.accepted
    assert res.r_trust == 0.8 * 2.0


def test_solved_step_is_accepted():
    prob = synth.config1()
    o = dr.Options(max_admm=200, max_dr=200, eps_kkt=1e-4, rho=200.0, sigma_s=10.0, cold_init="margin")
    res = scp.step(prob, prob.u_init, 2.0, "dr", o)
    assert res.info["status"] == "ok" and res.kkt <= 1e-4
    assert res.accepted
    assert res.r_trust >= 2.0
    # the merit model predicted a decrease and the nonlinear rollout realised at least a tenth of it
    assert res.merit_old - res.predicted > 0
    assert (res.merit_old - res.merit_new) >= 0.1 * (res.merit_old - res.predicted)
    assert np.linalg.norm(res.du) > 0
