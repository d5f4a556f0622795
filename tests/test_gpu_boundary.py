"""The C ABI's boundary on the GPU: nrto_solve_socp_dev on caller-owned device
buffers gives the solves of nrto_solve_socp on the same data (cold, then warm
from the returned state); the stop rule for infeasible linearisations returns
NRTO_INFEASIBLE at the oracle's ADMM iteration; NaN inputs propagate and are
flagged in the report."""
import numpy as np
import pytest

import synth
from oracle import dr, linearize

from helpers import compact_socp, rel_err

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


def test_device_buffer_solve_matches_context_solve():
    torch = _torch()
    from paper_2603_02642_amd import nrto
    pairs = [_near_obstacle(), _quad20()]
    probs = [p for p, _ in pairs]
    socps = [compact_socp(linearize.assemble(p, p.u_init, r)) for p, r in pairs]
    opt = lambda: nrto.default_options(method=0, max_admm=3, max_inner=10, eps_kkt=0.0, eps_dr_abs=0.0,
                                       eps_dr_rel=0.0, rho=50.0, sigma_s=100.0, cold_init=1, r_trust=2.0)
    ca = nrto.Context(probs, opt())
    cb = nrto.Context(probs, opt())
    for i, d in enumerate(socps):
        ca.upload_socp(i, **d)
    cat = lambda k: torch.from_numpy(np.concatenate([np.ravel(d[k]) for d in socps])).cuda()
    socp = {k: cat(k) for k in ("A", "B", "xhat", "uhat", "g0", "w", "bhat", "bvec")}
    sz = [ca.sizes(i) for i in range(2)]
    n = lambda f: sum(f(s) for s in sz)
    z = lambda m: torch.zeros(m, dtype=torch.float64, device="cuda")
    state = dict(st=z(n(lambda s: s["nent"])), kt=z(n(lambda s: s["T"] * s["nu"] * s["nx"])),
                 ptt=z(n(lambda s: s["ng"])), du=z(n(lambda s: s["T"] * s["nu"])),
                 K=z(n(lambda s: s["T"] * s["nu"] * s["nx"])), p=z(n(lambda s: s["ng"])),
                 pt=z(n(lambda s: s["ng"])), lam=z(n(lambda s: s["ng"])), pi=z(n(lambda s: s["ng"])))
    for warm in (False, True):
        print(f"device-buffer solve warm={warm}", flush=True)
        ra = ca.solve(warm=warm)
        rb = cb.solve_dev(socp, state, warm=warm)
        for i in range(2):
            assert ra[i].admm_iters == rb[i].admm_iters and ra[i].inner_iters == rb[i].inner_iters
            assert abs(ra[i].kkt - rb[i].kkt) <= 1e-9 * max(1.0, ra[i].kkt)
        offs = {}
        for key, f in (("st", lambda s: s["nent"]), ("kt", lambda s: s["T"] * s["nu"] * s["nx"]),
                       ("ptt", lambda s: s["ng"]), ("du", lambda s: s["T"] * s["nu"]),
                       ("K", lambda s: s["T"] * s["nu"] * s["nx"]), ("p", lambda s: s["ng"]),
                       ("pt", lambda s: s["ng"]), ("lam", lambda s: s["ng"]), ("pi", lambda s: s["ng"])):
            offs[key] = np.concatenate([[0], np.cumsum([f(s) for s in sz])])
        host = {k: v.cpu().numpy() for k, v in state.items()}
        for i in range(2):
            g, gs = ca.solution(i), ca.state(i)
            part = lambda k: host[k][offs[k][i]:offs[k][i + 1]]
            assert rel_err(part("du"), g["du"]) <= 1e-12
            assert rel_err(part("K"), g["K"].ravel()) <= 1e-12
            for k in ("p", "pt", "lam", "pi"):
                assert rel_err(part(k), g[k]) <= 1e-12, k
            assert rel_err(part("st"), gs["st"]) <= 1e-12
            assert rel_err(part("kt"), gs["kt"].ravel()) <= 1e-12
            assert rel_err(part("ptt"), gs["ptt"]) <= 1e-12


@pytest.mark.parametrize("r_trust,status", [(1e-3, "infeasible"), (5.0, "ok")])
def test_infeasible_linearisation_matches_oracle(r_trust, status):
    _torch()
    from paper_2603_02642_amd import nrto
    prob = synth.config1()
    prob.T = 8
    prob.radius = 0.02
    prob.u_init = np.tile([1.0, 0.0], (8, 1))
    prob.obstacles = np.array([[0.5, 0.04, 0.06]])
    s = linearize.assemble(prob, prob.u_init, r_trust)
    o = dr.Options(rho=50.0, sigma_s=10.0, cold_init="margin", max_admm=300, max_dr=100, eps_kkt=1e-4,
                   infeas_window=20)
    st, info = dr.solve(s, o)
    assert info["status"] == status
    c = nrto.Context([prob], nrto.default_options(method=0, max_admm=300, max_inner=100, eps_kkt=1e-4,
                                                  rho=50.0, sigma_s=10.0, cold_init=1, r_trust=r_trust,
                                                  infeas_window=20))
    c.upload_socp(0, **compact_socp(s))
    rep = c.solve()[0]
    print(f"infeasibility case r_trust={r_trust}: device status {rep.status} at {rep.admm_iters}, "
          f"oracle {info['status']} at {info['admm_iters']}", flush=True)
    want = nrto.NRTO_INFEASIBLE if status == "infeasible" else nrto.NRTO_OK
    assert rep.status == want
    assert rep.admm_iters == info["admm_iters"]
    assert rel_err(c.solution(0)["du"], st.du) <= 1e-6


def test_nan_input_is_flagged():
    _torch()
    from paper_2603_02642_amd import nrto
    prob, r = _near_obstacle()
    d = compact_socp(linearize.assemble(prob, prob.u_init, r))
    d["bhat"] = d["bhat"].copy()
    d["bhat"][5] = np.nan
    c = nrto.Context([prob], nrto.default_options(method=0, max_admm=20, max_inner=10, eps_kkt=1e-4, r_trust=r))
    c.upload_socp(0, **d)
    rep = c.solve()[0]
    assert rep.nan_flag == 1 and rep.status == nrto.NRTO_MAXITER
    d["bhat"][5] = 0.0
    c.upload_socp(0, **d)
    rep = c.solve()[0]
    assert rep.nan_flag == 0
