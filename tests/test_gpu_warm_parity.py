"""GPU parity of the learned-warm-start reconstruction (nrto_warm_start) with
the oracle's (oracle/warm.py) on the same SOCP and the same float32 prediction
rows (du, p~, pi): the rebuilt DR state element by element, the warm and cold
KKT residuals of the fallback test, and the fallback decision, for a
prediction taken from the oracle's converged solution, a perturbed one and a
bad one (which falls back to the cold point)."""
import numpy as np
import pytest

import synth
from oracle import dr, linearize, warm

from helpers import compact_socp, expand_entries, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _near_obstacle():
    prob = synth.config1()
    prob.T = 8
    prob.radius = 0.05
    prob.u_init = np.tile([1.0, 0.0], (8, 1))
    prob.obstacles = np.array([[0.45, 0.3, 0.15]])
    return prob, 5.0


def _quad20():
    prob = synth.config2()
    prob.T = 20
    prob.u_init = prob.u_init[:20]
    return prob, 2.0


@pytest.mark.parametrize("make", [_near_obstacle, _quad20])
@pytest.mark.parametrize("kind", ["converged", "perturbed", "bad"])
def test_warm_start_state_matches_oracle(make, kind):
    torch = _torch()
    from paper_2603_02642_amd import nrto
    prob, r = make()
    s = linearize.assemble(prob, prob.u_init, r)
    o = dr.Options(rho=50.0, sigma_s=100.0, cold_init="margin", max_admm=300, max_dr=100, eps_kkt=1e-6)
    sol, info = dr.solve(s, o)
    du, pt, pi = sol.du, sol.pt, sol.pi
    if kind == "perturbed":
        du = du + 0.05 * (2 * synth.uniform(21, du.size) - 1)
        pt = pt * (1 + 0.2 * (2 * synth.uniform(22, pt.size) - 1))
        pi = pi + 0.3 * (2 * synth.uniform(23, pi.size) - 1)
    elif kind == "bad":
        du = 40.0 * np.ones_like(du)
        pi = 100.0 * np.ones_like(pi)
    row = np.concatenate([du, pt, pi]).astype(np.float32)
    r64 = row.astype(np.float64)
    n_du = s.T * s.nu
    ref, keep, r_w, r_c = warm.warm_or_cold(s, o, r64[:n_du], r64[n_du:n_du + s.ng], r64[n_du + s.ng:])
    print(f"warm parity case {make.__name__} {kind}: oracle keep={keep} r_warm={r_w:.3e} r_cold={r_c:.3e}",
          flush=True)
    c = nrto.Context([prob], nrto.default_options(method=0, rho=50.0, sigma_s=100.0, cold_init=1, r_trust=r))
    c.upload_socp(0, **compact_socp(s))
    acc, res = c.warm_start(torch.from_numpy(row[None, :]).cuda(), fallback_test=True, gains=False)
    assert bool(acc[0]) == keep
    assert abs(res[0, 0] - r_w) <= 1e-9 * max(1.0, r_w)
    assert abs(res[0, 1] - r_c) <= 1e-9 * max(1.0, r_c)
    g = c.solution(0)
    gs = c.state(0)
    assert rel_err(g["du"], ref.du) <= 1e-12
    assert np.max(np.abs(g["K"])) == 0.0 and np.max(np.abs(gs["kt"])) == 0.0
    assert rel_err(g["p"], ref.p) <= 1e-12
    assert rel_err(g["pt"], ref.pt) <= 1e-12
    assert rel_err(gs["ptt"], ref.pt_t) <= 1e-12
    assert rel_err(g["lam"], ref.lam) <= 1e-12
    assert rel_err(expand_entries(s, gs["st"]), ref.s_t) <= 1e-12
    if keep:
        assert rel_err(g["pi"], ref.pi) <= 1e-12
    c.close()
