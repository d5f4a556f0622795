"""NRTO-DR: the inner ADMM of NRTO with its {k_v, p~} block solved by relaxed
Douglas-Rachford splitting (Section III; supplementary section II).

ADMM (the three updates of Section II-B; the dual update uses the current
p - p~, a reading of the printed superscripts):
    {k_v, p~} <- DR solve of the subproblem (eq. dr-subproblem)
    {du, p}   <- oracle.qp with c = p~ - lambda / rho
    lambda    <- lambda + rho (p - p~)

DR on min 1/2 chi'P chi + q'chi s.t. A chi + s = b, s in K, chi = [k_v; p~],
P = blkdiag(Q_v, rho I), q = [0; -(rho p + lambda)], s_j = (t_j, eta_j),
t_j = p~_j, eta_j = A_hat_j k_v + b_hat_j (supplementary II-A):
    xi       = Prox_J(xi~)                 affine-set prox, R_chi = sigma_chi I,
                                           R_s = sigma_s I; y eliminated, so the
                                           k_v block is solved with
                                           H = Q_v + sigma_chi I + sigma_s sum_j A_hat_j'A_hat_j
                                           (dense Cholesky, factored once) and
                                           s = b - A chi
    xi_ref   = 2 xi - xi~
    xi~     += alpha (Prox_Jhat(xi_ref) - xi),  Prox_Jhat = (identity on chi, Pi_K on s)
stopped when ||s~_new - s~_old||_2 <= eps_abs + eps_rel max(1, ||s~||) or after
max_dr steps.  The DR state xi~ is carried from one ADMM iteration to the next.

Two options depart from the printed method (both off by default):
  cold_init = "margin": the cold point starts every cone at its open-loop value,
    p = p~ = p~~ = ||b_hat_j||, s~_j = (||b_hat_j||, b_hat_j), so that k_v = 0 is
    feasible for every cone; the printed initialisation is all zeros.  From
    zeros, a cone whose constraint is slack still holds p~ below ||b_hat_j|| and
    the only force lifting it is the proximal term rho/2 ||p~ - p||^2, which
    moves it by O(1/rho) per ADMM iteration (sublinear creep).
  rho_adapt: residual balancing of the penalty (Boyd et al., Foundations and
    Trends in ML 3(1), 2011, section 3.4.1): after the dual update, rho <- rho
    tau when r_p > mu r_d, rho <- rho / tau when r_d > mu r_p, kept in
    [rho_min, rho_max].  lambda is unscaled, so it is kept as it is; the
    k_v factor does not involve rho, so nothing is refactored.
  infeas_window (a reading; the paper notes only that linearised problems can
    be infeasible): stop with status "infeasible" when r_p = ||p - p~|| has not
    fallen below 0.99 times its smallest earlier value for infeas_window ADMM
    iterations while r_p / (1 + ||p~||) > 1e-3.
  sigma_adapt: balancing of the DR scaling sigma_s (in the spirit of OSQP's
    step-size rule, Stellato et al., Math. Prog. Comp. 12, 2020): after every
    sigma_every-th DR iteration of a solve, with S = (p~, eta(K)) the affine
    point, S_hat its projection, K~ the gain state before the iteration,
      r_prim = ||S_hat - S||,  r_dual = ||K - K~||,
      ratio = sqrt((r_prim / max(1, ||S||)) / (r_dual / max(1, ||K||))),
    sigma_s <- clip(sigma_s ratio, sigma_min, sigma_max) when ratio > sigma_thr
    or ratio < 1 / sigma_thr; residuals at rounding level (r_prim <=
    1e-9 max(1, ||S||) or r_dual <= 1e-9 max(1, ||K||)) leave sigma_s as it is.  The cone state keeps its multiplier estimate:
    s~ <- S + (sigma_old / sigma_new)(s~ - S); the k_v blocks are refactored.
    With every cone slack, the DR iteration contracts K towards its minimiser
    by (sigma_chi + sigma_s l)/(q + sigma_chi + sigma_s l) along an eigenvector
    of sum_j A_hat_j'A_hat_j with eigenvalue l (q: the curvature of Q_v), so a
    sigma_s fit for the active cones can stall the gains; the rule moves it.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla

from . import kkt, qp
from .linearize import AtA_dense, K_to_kv, Qv_dense, eta, eta_adjoint, kv_to_K
from .soc import project_rows_vec


@dataclasses.dataclass
class Options:
    rho: float = 40.0
    alpha: float = 1.0
    sigma_chi: float = 1.0
    sigma_s: float = 1.0
    eps_dr_abs: float = 1e-4
    eps_dr_rel: float = 1e-4
    max_dr: int = 100
    max_admm: int = 40
    eps_kkt: float = 1e-4
    check_every: int = 1
    eps_p: float = 0.0
    eps_d: float = 0.0
    cold_init: str = "zero"        # "zero" (printed) or "margin"
    rho_adapt: bool = False
    rho_mu: float = 10.0
    rho_tau: float = 2.0
    rho_min: float = 1.0
    rho_max: float = 200.0
    sigma_adapt: bool = False
    sigma_every: int = 10
    sigma_thr: float = 5.0
    sigma_min: float = 1e-4
    sigma_max: float = 1e6
    infeas_window: int = 0          # 0 = off (see solve)


@dataclasses.dataclass
class State:
    K_t: np.ndarray      # K~   (T, nu, nx)
    pt_t: np.ndarray     # p~~  (ng,)
    s_t: np.ndarray      # s~   (ng, 1 + nz): column 0 = t, then eta
    du: np.ndarray
    p: np.ndarray
    lam: np.ndarray
    K: np.ndarray        # last chi (k_v part)
    pt: np.ndarray       # last chi (p~ part)
    pi: np.ndarray
    mu: float
    sigma_s: Optional[float] = None   # current DR scaling (None: the option's)


def zero_state(socp) -> State:
    T, nu, nx, ng = socp.T, socp.nu, socp.nx, socp.ng
    return State(K_t=np.zeros((T, nu, nx)), pt_t=np.zeros(ng), s_t=np.zeros((ng, 1 + socp.nz)),
                 du=np.zeros(T * nu), p=np.zeros(ng), lam=np.zeros(ng),
                 K=np.zeros((T, nu, nx)), pt=np.zeros(ng), pi=np.zeros(ng), mu=0.0)


def cold_state(socp, opt: Options) -> State:
    """The cold point: zeros, or with cold_init == "margin" every cone at its
    open-loop value (||b_hat_j||, b_hat_j) with p = p~ = p~~ = ||b_hat_j||."""
    st = zero_state(socp)
    if opt.cold_init == "margin":
        nb = np.sqrt(np.sum(socp.bhat * socp.bhat, axis=1))
        st.p[:] = nb
        st.pt[:] = nb
        st.pt_t[:] = nb
        st.s_t[:, 0] = nb
        st.s_t[:, 1:] = socp.bhat
    elif opt.cold_init != "zero":
        raise ValueError(opt.cold_init)
    return st


def _sigma(opt: Options, st: State) -> float:
    return opt.sigma_s if st.sigma_s is None else st.sigma_s


def zeta(socp, opt: Options, st: State) -> np.ndarray:
    """Cone multiplier y_eta = sigma_s (eta~ - eta(K)) of the affine-set prox."""
    return _sigma(opt, st) * (st.s_t[:, 1:] - eta(socp, st.K))


def residual(socp, opt: Options, st: State) -> float:
    return kkt.residual(socp, st.du, st.K, st.p, st.pt, st.pi, st.mu, zeta(socp, opt, st))


def factor(socp, opt: Options, sigma_s: Optional[float] = None):
    n = socp.T * socp.nu * socp.nx
    ss = opt.sigma_s if sigma_s is None else sigma_s
    Hk = Qv_dense(socp) + opt.sigma_chi * np.eye(n) + ss * AtA_dense(socp)
    return sla.cho_factor(Hk, lower=True)


def dr_steps(socp, opt: Options, st: State, fac, max_steps: int, trace: Optional[Callable] = None,
             n_done: int = 0):
    """Run up to max_steps relaxed DR iterations on the current subproblem.
    n_done: DR iterations of this solve so far (sigma_adapt acts after every
    sigma_every-th).  Returns (steps, r_dr, fac) -- fac is refactored when
    sigma_s changes."""
    rho, al, sx = opt.rho, opt.alpha, opt.sigma_chi
    ss = _sigma(opt, st)
    T, nu, nx = socp.T, socp.nu, socp.nx
    r_dr = np.inf
    it = 0
    for it in range(1, max_steps + 1):
        # Prox_J: reduced KKT solve
        R = sx * st.K_t + ss * eta_adjoint(socp, st.s_t[:, 1:] - socp.bhat)
        K = kv_to_K(sla.cho_solve(fac, K_to_kv(R)), T, nu, nx)
        pt = (sx * st.pt_t + rho * st.p + st.lam + ss * st.s_t[:, 0]) / (rho + sx + ss)
        S = np.empty_like(st.s_t)
        S[:, 0] = pt
        S[:, 1:] = eta(socp, K)
        # reflection, cone prox, relaxation
        S_ref = 2.0 * S - st.s_t
        S_hat = project_rows_vec(S_ref)
        dK = K - st.K_t
        st.K_t = st.K_t + al * dK
        st.pt_t = st.pt_t + al * (pt - st.pt_t)
        dS = al * (S_hat - S)
        st.s_t = st.s_t + dS
        st.K, st.pt = K, pt
        r_dr = float(np.sqrt(np.sum(dS * dS)))
        if opt.sigma_adapt and (n_done + it) % opt.sigma_every == 0:
            n_s = max(1.0, float(np.sqrt(np.sum(S * S))))
            n_k = max(1.0, float(np.sqrt(np.sum(K * K))))
            r_prim = r_dr / al
            r_dual = float(np.sqrt(np.sum(dK * dK)))
            if r_prim > 1e-9 * n_s and r_dual > 1e-9 * n_k:
                ratio = np.sqrt((r_prim / n_s) / (r_dual / n_k))
                if ratio > opt.sigma_thr or ratio < 1.0 / opt.sigma_thr:
                    new = min(max(ss * ratio, opt.sigma_min), opt.sigma_max)
                    if new != ss:
                        st.sigma_updates = getattr(st, "sigma_updates", 0) + 1
                        st.s_t = S + (ss / new) * (st.s_t - S)
                        ss = new
                        st.sigma_s = ss
                        fac = factor(socp, opt, ss)
        if trace is not None:
            trace("dr", it, st)
        if r_dr <= opt.eps_dr_abs + opt.eps_dr_rel * max(1.0, float(np.sqrt(np.sum(st.s_t * st.s_t)))):
            break
    return it, r_dr, fac


def solve(socp, opt: Options = Options(), st: Optional[State] = None, trace: Optional[Callable] = None):
    """Returns (State, info dict)."""
    opt = dataclasses.replace(opt)      # rho_adapt changes opt.rho
    if st is None:
        st = cold_state(socp, opt)
    if st.sigma_s is None:
        st.sigma_s = opt.sigma_s
    fac = factor(socp, opt, st.sigma_s)
    info = {"admm_iters": 0, "dr_iters": 0, "kkt": np.inf, "status": "maxiter", "r_p": np.inf, "r_d": np.inf}
    pt_prev = st.pt.copy()
    rp_best, l_best = np.inf, 0
    for l in range(1, opt.max_admm + 1):
        n_dr, _, fac = dr_steps(socp, opt, st, fac, opt.max_dr, trace, info["dr_iters"])
        info["dr_iters"] += n_dr
        c = st.pt - st.lam / opt.rho
        st.du, st.p, st.pi, st.mu = qp.solve(socp.H, socp.h, socp.bmat, socp.g0, c, opt.rho,
                                             socp.Fu, socp.r_trust, st.du)
        st.lam = st.lam + opt.rho * (st.p - st.pt)
        info["admm_iters"] = l
        info["r_p"] = float(np.linalg.norm(st.p - st.pt))
        info["r_d"] = float(opt.rho * np.linalg.norm(st.pt - pt_prev))
        pt_prev = st.pt.copy()
        if trace is not None:
            trace("admm", l, st)
        stop = False
        if opt.eps_kkt > 0 and (l % opt.check_every == 0 or l == opt.max_admm):
            info["kkt"] = residual(socp, opt, st)
            stop = info["kkt"] <= opt.eps_kkt
        if opt.eps_p > 0 and opt.eps_d > 0 and info["r_p"] <= opt.eps_p and info["r_d"] <= opt.eps_d:
            stop = True
        if stop:
            info["status"] = "ok"
            break
        if opt.infeas_window > 0:
            # the linearised problem may be infeasible (e.g. inside a small trust
            # region): then ADMM's consensus residual stalls at the sets' distance
            if info["r_p"] < 0.99 * rp_best:
                rp_best, l_best = info["r_p"], l
            if l - l_best >= opt.infeas_window and info["r_p"] > 1e-3 * (1.0 + float(np.linalg.norm(st.pt))):
                info["status"] = "infeasible"
                break
        if opt.rho_adapt:
            if info["r_p"] > opt.rho_mu * info["r_d"]:
                opt.rho = min(opt.rho_max, opt.rho * opt.rho_tau)
            elif info["r_d"] > opt.rho_mu * info["r_p"]:
                opt.rho = max(opt.rho_min, opt.rho / opt.rho_tau)
    info["kkt"] = residual(socp, opt, st)
    info["rho"] = opt.rho
    info["sigma_s"] = st.sigma_s
    info["sigma_updates"] = getattr(st, "sigma_updates", 0)
    return st, info
