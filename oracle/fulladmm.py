"""NRTO-FullADMM (Section IV, Algorithm 1; supplementary section III).

Slack nu_j = A_hat_j k_v + b_hat_j with ||nu_j|| <= p~_j and p = p~; blocks
(nu, p~) and (du, p, k_v); scaled duals lambda_p, lambda_nu (dual variables
rho lambda_p, rho lambda_nu).  One iteration, in the paper's order:

  Block 1   (nu_j, p~_j) = Pi_SOC(A_hat_j k_v + b_hat_j + lambda_nu_j,  p_j + lambda_p_j)
  Block 2a  (du, p)      = oracle.qp with c = p~ - lambda_p
  Block 2b  k_v          = M (Q_v k_v^- + rho sum_j A_hat_j'(nu_j - b_hat_j)),
                           M = (Q_v + rho sum_j A_hat_j'A_hat_j)^-1  (the closed form
                           q + calM k_v^- + calMbar nu; "b_j" there read as b_hat_j)
  Dual      lambda_p += p - p~ ;  lambda_nu_j += A_hat_j k_v + b_hat_j - nu_j

Initialisation at zero keeps Q_v k_v + rho sum_j A_hat_j' lambda_nu_j = 0, the
invariant the closed form relies on.  Stopping: the KKT residual (every
`check_every` iterations) and optionally r_p = ||p - p~||, r_d = rho ||p~ - p~_prev||
together with r_nu = ||A_hat k_v + b_hat - nu||.
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
    rho: float = 10.0
    max_admm: int = 40
    eps_kkt: float = 1e-4
    check_every: int = 1
    eps_p: float = 0.0
    eps_d: float = 0.0
    eps_nu: float = 0.0


@dataclasses.dataclass
class State:
    K: np.ndarray        # (T, nu, nx)
    nu_: np.ndarray      # (ng, nz)
    pt: np.ndarray       # p~
    du: np.ndarray
    p: np.ndarray
    lam_p: np.ndarray
    lam_nu: np.ndarray   # (ng, nz)
    pi: np.ndarray
    mu: float


def zero_state(socp) -> State:
    T, nu, nx, ng, nz = socp.T, socp.nu, socp.nx, socp.ng, socp.nz
    return State(K=np.zeros((T, nu, nx)), nu_=np.zeros((ng, nz)), pt=np.zeros(ng),
                 du=np.zeros(T * nu), p=np.zeros(ng), lam_p=np.zeros(ng),
                 lam_nu=np.zeros((ng, nz)), pi=np.zeros(ng), mu=0.0)


def residual(socp, opt: Options, st: State) -> float:
    """KKT residual with the cone multiplier zeta = -rho lambda_nu."""
    return kkt.residual(socp, st.du, st.K, st.p, st.pt, st.pi, st.mu, -opt.rho * st.lam_nu)


def factor(socp, opt: Options):
    return sla.cho_factor(Qv_dense(socp) + opt.rho * AtA_dense(socp), lower=True)


def invariant(socp, opt: Options, st: State) -> np.ndarray:
    """Q_v k_v + rho sum_j A_hat_j' lambda_nu_j as an array (T, nu, nx)."""
    qk = 2.0 * np.einsum("uv,kvx->kux", socp.RK2, st.K)
    return qk + opt.rho * eta_adjoint(socp, st.lam_nu)


def iterate(socp, opt: Options, st: State, fac):
    """One FullADMM iteration; returns (r_p, r_d, r_nu)."""
    rho = opt.rho
    T, nu, nx = socp.T, socp.nu, socp.nx
    # Block 1
    a = eta(socp, st.K)
    S = np.empty((socp.ng, 1 + socp.nz))
    S[:, 0] = st.p + st.lam_p
    S[:, 1:] = a + st.lam_nu
    P = project_rows_vec(S)
    pt_prev = st.pt
    st.pt = P[:, 0].copy()
    st.nu_ = P[:, 1:].copy()
    # Block 2a
    c = st.pt - st.lam_p
    st.du, st.p, st.pi, st.mu = qp.solve(socp.H, socp.h, socp.bmat, socp.g0, c, rho,
                                         socp.Fu, socp.r_trust, st.du)
    # Block 2b (closed form)
    rhs = 2.0 * np.einsum("uv,kvx->kux", socp.RK2, st.K) + rho * eta_adjoint(socp, st.nu_ - socp.bhat)
    st.K = kv_to_K(sla.cho_solve(fac, K_to_kv(rhs)), T, nu, nx)
    # duals
    st.lam_p = st.lam_p + (st.p - st.pt)
    a_new = eta(socp, st.K)
    st.lam_nu = st.lam_nu + (a_new - st.nu_)
    # the stationarity multiplier of g0 + B du + p <= 0 is -rho lambda_p after the update
    r_p = float(np.linalg.norm(st.p - st.pt))
    r_d = float(rho * np.linalg.norm(st.pt - pt_prev))
    r_nu = float(np.linalg.norm(a_new - st.nu_))
    return r_p, r_d, r_nu


def solve(socp, opt: Options = Options(), st: Optional[State] = None, trace: Optional[Callable] = None):
    if st is None:
        st = zero_state(socp)
    fac = factor(socp, opt)
    info = {"admm_iters": 0, "kkt": np.inf, "status": "maxiter"}
    for l in range(1, opt.max_admm + 1):
        r_p, r_d, r_nu = iterate(socp, opt, st, fac)
        info.update(admm_iters=l, r_p=r_p, r_d=r_d, r_nu=r_nu)
        if trace is not None:
            trace("admm", l, st)
        stop = False
        if opt.eps_kkt > 0 and (l % opt.check_every == 0):
            info["kkt"] = residual(socp, opt, st)
            stop = info["kkt"] <= opt.eps_kkt
        if opt.eps_p > 0 and r_p <= opt.eps_p and r_d <= opt.eps_d and r_nu <= max(opt.eps_nu, 0.0):
            stop = True
        if stop:
            info["status"] = "ok"
            break
    info["kkt"] = residual(socp, opt, st)
    return st, info
