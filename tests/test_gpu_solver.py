"""GPU parity of the persistent solver against the oracle on the same SOCP
data (produced by the oracle, marshalled into the compact layout):
iterates after fixed iteration counts (no early stop) within 1e-9 relative in
FP64, and the converged solves reaching the 1e-4 KKT residual."""
import numpy as np
import pytest

import synth
from oracle import dr, fulladmm, kkt, linearize

from helpers import compact_socp, expand_entries, rel_err

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def near_obstacle_problem(T=8, radius=0.05):
    prob = synth.config1()
    prob.T = T
    prob.radius = radius
    prob.u_init = np.tile([1.0, 0.0], (T, 1))
    prob.obstacles = np.array([[0.45, 0.3, 0.15]])
    return prob


def _ctx(prob, s, **opt):
    from paper_2603_02642_amd import nrto
    o = nrto.default_options(**opt)
    c = nrto.Context([prob], o)
    c.upload_socp(0, **compact_socp(s))
    return c


@pytest.mark.parametrize("T,L,M,alpha,extra", [(8, 3, 15, 1.0, {}), (8, 2, 10, 1.6, {}), (6, 2, 10, 0.5, {}),
                                               (8, 8, 10, 1.0, {"cold_init": 1, "rho_adapt": 1}),
                                               (7, 6, 12, 1.2, {"rho_adapt": 1, "rho": 200.0, "sigma_s": 10.0}),
                                               (8, 6, 10, 1.0, {"cold_init": 1, "rho": 200.0, "sigma_s": 100.0,
                                                                "sigma_adapt": 1, "sigma_every": 3,
                                                                "sigma_thr": 1.2})])
def test_dr_iterates_match_oracle_fp64(T, L, M, alpha, extra):
    _torch()
    prob = near_obstacle_problem(T)
    s = linearize.assemble(prob, prob.u_init, 5.0)
    ox = dict(rho=extra.get("rho", 40.0), sigma_s=extra.get("sigma_s", 1.0))
    sx = dict(sigma_every=extra.get("sigma_every", 10), sigma_thr=extra.get("sigma_thr", 5.0))
    o = dr.Options(max_admm=L, max_dr=M, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0, alpha=alpha,
                   cold_init="margin" if extra.get("cold_init") else "zero",
                   rho_adapt=bool(extra.get("rho_adapt")), sigma_adapt=bool(extra.get("sigma_adapt")), **sx, **ox)
    st, info = dr.solve(s, o)
    c = _ctx(prob, s, method=0, max_admm=L, max_inner=M, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0,
             alpha=alpha, r_trust=5.0, cold_init=extra.get("cold_init", 0), rho_adapt=extra.get("rho_adapt", 0),
             sigma_adapt=extra.get("sigma_adapt", 0), **sx, **ox)
    rep = c.solve()
    g = c.solution(0)
    gs = c.state(0)
    assert rep[0].admm_iters == L and rep[0].inner_iters == L * M
    assert rep[0].rho == info["rho"]
    if extra.get("rho_adapt"):
        assert info["rho"] != ox["rho"]        # the balancing acted within L iterations
    assert rep[0].sigma_updates == info["sigma_updates"]
    assert abs(rep[0].sigma_s - info["sigma_s"]) <= 1e-9 * info["sigma_s"]
    if extra.get("sigma_adapt"):
        assert info["sigma_s"] != ox["sigma_s"]
    assert rel_err(g["du"], st.du) <= 1e-9
    assert rel_err(g["K"], st.K) <= 1e-9
    assert rel_err(g["p"], st.p) <= 1e-9
    assert rel_err(g["pt"], st.pt) <= 1e-9
    assert rel_err(g["lam"], st.lam) <= 1e-9
    assert rel_err(expand_entries(s, gs["st"]), st.s_t) <= 1e-9
    assert rel_err(gs["kt"], st.K_t) <= 1e-9
    ref_kkt = dr.residual(s, o, st)
    assert abs(rep[0].kkt - ref_kkt) <= 1e-9 * max(1.0, ref_kkt)


FA_OFF = ("FullADMM device path switched off: its kernel took a GPU memory fault "
          "(aperture violation) whose cause is not yet identified")


@pytest.mark.skip(reason=FA_OFF)
@pytest.mark.parametrize("T,L", [(8, 30), (5, 12)])
def test_fulladmm_iterates_match_oracle_fp64(T, L):
    _torch()
    prob = near_obstacle_problem(T)
    s = linearize.assemble(prob, prob.u_init, 5.0)
    o = fulladmm.Options(max_admm=L, eps_kkt=0.0)
    st, _ = fulladmm.solve(s, o)
    c = _ctx(prob, s, method=1, max_admm=L, eps_kkt=0.0, rho=10.0, r_trust=5.0)
    rep = c.solve()
    g = c.solution(0)
    gs = c.state(0)
    assert rel_err(g["du"], st.du) <= 1e-9
    assert rel_err(g["K"], st.K) <= 1e-9
    assert rel_err(g["p"], st.p) <= 1e-9
    assert rel_err(g["pt"], st.pt) <= 1e-9
    assert rel_err(g["lam"], st.lam_p) <= 1e-9
    assert rel_err(expand_entries(s, gs["st"])[:, 1:], st.lam_nu) <= 1e-9
    assert rel_err(expand_entries(s, gs["nu"])[:, 1:], st.nu_) <= 1e-9
    ref_kkt = fulladmm.residual(s, o, st)
    assert abs(rep[0].kkt - ref_kkt) <= 1e-9 * max(1.0, ref_kkt)


def test_dr_long_cones_with_sigma_balancing_match_oracle():
    """Quadrotor (cones up to 253 entries: one wave per cone, two passes) with the
    DR scaling balanced every third iteration."""
    _torch()
    prob = synth.config2()
    prob.T = 20
    prob.u_init = prob.u_init[:20]
    s = linearize.assemble(prob, prob.u_init, 2.0)
    kw = dict(rho=200.0, sigma_s=100.0, sigma_every=3, sigma_thr=1.2)
    o = dr.Options(max_admm=3, max_dr=8, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0, sigma_adapt=True, **kw)
    st, info = dr.solve(s, o)
    assert info["sigma_s"] != 100.0
    c = _ctx(prob, s, method=0, max_admm=3, max_inner=8, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0,
             r_trust=2.0, sigma_adapt=1, **kw)
    rep = c.solve()
    g = c.solution(0)
    gs = c.state(0)
    assert abs(rep[0].sigma_s - info["sigma_s"]) <= 1e-9 * info["sigma_s"]
    assert rel_err(g["du"], st.du) <= 1e-9
    assert rel_err(g["K"], st.K) <= 1e-9
    assert rel_err(expand_entries(s, gs["st"]), st.s_t) <= 1e-9
    assert rel_err(gs["kt"], st.K_t) <= 1e-9


def test_trust_region_active_matches_oracle():
    _torch()
    prob = synth.config1()
    s = linearize.assemble(prob, prob.u_init, 2.0)
    o = dr.Options(max_admm=4, max_dr=20, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0)
    st, _ = dr.solve(s, o)
    assert st.mu > 0
    c = _ctx(prob, s, method=0, max_admm=4, max_inner=20, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0,
             r_trust=2.0)
    c.solve()
    g = c.solution(0)
    assert abs(g["mu"] - st.mu) <= 1e-9 * max(1.0, st.mu)
    assert rel_err(g["du"], st.du) <= 1e-9


def test_fulladmm_path_raises_while_switched_off():
    _torch()
    from paper_2603_02642_amd import nrto
    prob = near_obstacle_problem(5)
    c = nrto.Context([prob], nrto.default_options(method=1))
    with pytest.raises(nrto.NrtoError):
        c.solve()


def test_captured_step_replays_match_eager():
    """Linearise + solve captured in a HIP graph: every replay, with eager work
    and synchronisations in between, equals the eager result."""
    torch = _torch()
    from paper_2603_02642_amd import nrto
    probs = [synth.config4_instance(i) for i in (0, 1, 1024, 1025)]
    o = nrto.default_options(method=0, max_admm=3, max_inner=10, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0,
                             cold_init=1, rho=200.0, sigma_s=100.0, sigma_adapt=1, sigma_thr=2.0)
    stream = torch.cuda.Stream()
    c = nrto.Context(probs, o, stream=stream.cuda_stream)
    c.linearize()
    c.solve()
    ref = [c.solution(i) for i in range(len(probs))]
    c.capture_step(warm=False, with_linearize=True)
    for _ in range(3):
        c.launch_step()
        torch.cuda.synchronize()
        rep = c.reports()
        assert all(r.admm_iters == 3 for r in rep)
        for i in range(len(probs)):
            g = c.solution(i)
            assert rel_err(g["du"], ref[i]["du"]) <= 1e-9
            assert rel_err(g["K"], ref[i]["K"]) <= 1e-9
        c.linearize()            # eager work between replays
        c.solve()
        torch.cuda.synchronize()
    c.set_options(o)             # drops the captured step
    with pytest.raises(nrto.NrtoError):
        c.launch_step()


@pytest.mark.parametrize("L,M,policy", [(3, 10, False), (4, 12, True)])
def test_arm_dr_iterates_match_oracle_fp64(L, M, policy):
    """The 7-DOF arm (n_x = 14, n_u = 7, four obstacles tested at seven link
    points, joint and torque bounds) on a short horizon: fixed-count iterates of
    the device solver against the oracle, with the zero starting point or with
    the margin starting point and sigma_s balancing."""
    _torch()
    prob = synth.config3()
    prob.T = 6
    prob.u_init = prob.u_init[:6]
    s = linearize.assemble(prob, prob.u_init, 5.0)
    if policy:
        ox = dict(rho=50.0, sigma_s=100.0, sigma_every=3, sigma_thr=1.2)
        o = dr.Options(max_admm=L, max_dr=M, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0, cold_init="margin",
                       sigma_adapt=True, **ox)
        extra = dict(cold_init=1, sigma_adapt=1, **ox)
    else:
        o = dr.Options(max_admm=L, max_dr=M, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0, rho=40.0, sigma_s=1.0)
        extra = dict(rho=40.0, sigma_s=1.0)
    st, info = dr.solve(s, o)
    c = _ctx(prob, s, method=0, max_admm=L, max_inner=M, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0,
             r_trust=5.0, **extra)
    rep = c.solve()
    g = c.solution(0)
    assert rep[0].admm_iters == L and rep[0].inner_iters == L * M
    assert rep[0].sigma_updates == info["sigma_updates"]
    for k in ["du", "K", "p", "pt", "lam"]:
        assert rel_err(g[k], getattr(st, k)) <= 1e-9, k
    ref_kkt = dr.residual(s, o, st)
    assert abs(rep[0].kkt - ref_kkt) <= 1e-9 * max(1.0, ref_kkt)


BENCH = dict(rho=50.0, sigma_s=100.0, sigma_every=10, sigma_thr=2.0)


def test_full_size_quadrotor_iterates_at_bench_settings():
    """The quadrotor at its full horizon (T = 50, five obstacles, thrust bounds:
    cones up to 613 entries) under the benchmark's solver settings (rho 50,
    sigma_s from 100 balanced every 10 DR iterations with threshold 2, margin
    start): fixed-count DR iterates against the oracle at 1e-9."""
    _torch()
    prob = synth.config2()
    s = linearize.assemble(prob, prob.u_init, 2.0)
    o = dr.Options(max_admm=3, max_dr=15, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0, cold_init="margin",
                   sigma_adapt=True, **BENCH)
    st, info = dr.solve(s, o)
    print(f"full-size quadrotor: oracle sigma updates {info['sigma_updates']}", flush=True)
    c = _ctx(prob, s, method=0, max_admm=3, max_inner=15, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0,
             r_trust=2.0, cold_init=1, sigma_adapt=1, **BENCH)
    rep = c.solve()
    g = c.solution(0)
    gs = c.state(0)
    assert rep[0].sigma_updates == info["sigma_updates"]
    for k in ["du", "K", "p", "pt", "lam"]:
        assert rel_err(g[k], getattr(st, k)) <= 1e-9, k
    assert rel_err(expand_entries(s, gs["st"]), st.s_t) <= 1e-9
    assert rel_err(gs["kt"], st.K_t) <= 1e-9
    ref_kkt = dr.residual(s, o, st)
    assert abs(rep[0].kkt - ref_kkt) <= 1e-9 * max(1.0, ref_kkt)


def test_full_size_arm_iterates_match_oracle():
    """The 7-DOF arm at its full horizon (T = 60: 3360 cones, 1.1 million cone
    entries, LDS of one instance near the compute unit's 160 KB) with the
    margin start and sigma_s balancing: fixed-count DR iterates at 1e-9."""
    _torch()
    prob = synth.config3()
    s = linearize.assemble(prob, prob.u_init, 5.0)
    ox = dict(rho=50.0, sigma_s=100.0, sigma_every=3, sigma_thr=1.2)
    o = dr.Options(max_admm=2, max_dr=4, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0, cold_init="margin",
                   sigma_adapt=True, **ox)
    st, info = dr.solve(s, o)
    c = _ctx(prob, s, method=0, max_admm=2, max_inner=4, eps_kkt=0.0, eps_dr_abs=0.0, eps_dr_rel=0.0,
             r_trust=5.0, cold_init=1, sigma_adapt=1, **ox)
    rep = c.solve()
    g = c.solution(0)
    gs = c.state(0)
    assert rep[0].sigma_updates == info["sigma_updates"]
    for k in ["du", "K", "p", "pt", "lam"]:
        assert rel_err(g[k], getattr(st, k)) <= 1e-9, k
    assert rel_err(expand_entries(s, gs["st"]), st.s_t) <= 1e-9
    ref_kkt = dr.residual(s, o, st)
    assert abs(rep[0].kkt - ref_kkt) <= 1e-9 * max(1.0, ref_kkt)
