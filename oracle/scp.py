"""Minimal successive-linearisation (SL / SCP) loop around the robust SOCP solve.

The paper's outer loop (trust-region acceptance, rho schedule, NRTO-LE) is
defined in its companion reference, which is not available; this is a plain
trust-region reading of the outer-loop hyperparameter tables (r_0 = 2,
r_min = 1e-3, shrink 0.8 / grow 1.5, penalty weight w_p = 10):

  merit(current)   = J(u_hat)            + w_p sum_j max(0, g0_j + n_j)
  merit(predicted) = Q_u(du)             + w_p sum_j max(0, g0_j + b_j' du + n_j)
  merit(actual)    = J(u_hat + du)       + w_p sum_j max(0, g_j(x(u_hat + du)) + n_j)

where J is the nominal cost on the nonlinear rollout, Q_u its linearisation,
n_j = ||A_hat_j k_v + b_hat_j|| the robust margin of the new gains (the same
in all three, so the ratio measures how well the linearised nominal
trajectory predicts the nonlinear one).  ratio = (cur - act) / (cur - pred);
accept if the inner solve reached its tolerance, the predicted decrease is
positive and ratio >= 0.1 (a step whose SOCP was not solved is never taken: its
du is not the minimiser the ratio test presumes); on acceptance
u_hat += du and the radius grows by 1.5 when ratio >= 0.75; on rejection it
shrinks by 0.8 (not below r_min).  Parity unpinned beyond the GPU comparison:
the paper prints no outer-loop trace.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import dr, fulladmm, linearize

W_P = 10.0
ETA_ACCEPT = 0.1
ETA_GROW = 0.75
SHRINK = 0.8
GROW = 1.5
R_MIN = 1e-3
R_MAX = 1e3


def nominal_cost(prob, u):
    x = linearize.rollout(prob, u)
    J = float(np.sum((u @ prob.Ru) * u))
    dev = x[1:] - prob.xg[None, :]
    J += float(np.sum((dev @ prob.Q) * dev))
    return J, x


def constraint_values(prob, x, u):
    """g_j at the trajectory (x, u), canonical constraint order."""
    vals = []
    for t in range(1, prob.T + 1):
        for (gv, _w) in linearize.state_constraints_at(prob, x[t]):
            vals.append(gv)
    for k in range(prob.T):
        for i in range(prob.nu):
            if prob.u_hi is not None and np.isfinite(prob.u_hi[i]):
                vals.append(u[k, i] - prob.u_hi[i])
            if prob.u_lo is not None and np.isfinite(prob.u_lo[i]):
                vals.append(prob.u_lo[i] - u[k, i])
    return np.array(vals)


@dataclasses.dataclass
class StepResult:
    accepted: bool
    merit_old: float
    merit_new: float
    predicted: float
    r_trust: float
    kkt: float
    du: np.ndarray
    K: np.ndarray
    info: dict = dataclasses.field(default_factory=dict)


def step(prob, uhat, r_trust, method="dr", opt=None):
    s = linearize.assemble(prob, uhat, r_trust)
    if method == "dr":
        opt = opt or dr.Options()
        st, info = dr.solve(s, opt)
    else:
        opt = opt or fulladmm.Options()
        st, info = fulladmm.solve(s, opt)
    du, K = st.du, st.K
    E = linearize.eta(s, K)
    n = np.sqrt(np.sum(E * E, axis=1))
    J0, _ = nominal_cost(prob, uhat)
    cur = J0 + W_P * float(np.sum(np.maximum(0.0, s.g0 + n)))
    pred = linearize.qu_value(s, du) + W_P * float(np.sum(np.maximum(0.0, s.g0 + s.bmat @ du + n)))
    unew = uhat + du.reshape(prob.T, prob.nu)
    J1, x1 = nominal_cost(prob, unew)
    g1 = constraint_values(prob, x1, unew)
    act = J1 + W_P * float(np.sum(np.maximum(0.0, g1 + n)))
    dpred = cur - pred
    ratio = (cur - act) / dpred if dpred > 0 else -np.inf
    accepted = bool(info["status"] == "ok" and dpred > 0 and ratio >= ETA_ACCEPT)
    if accepted:
        r_new = min(GROW * r_trust, R_MAX) if ratio >= ETA_GROW else r_trust
    else:
        r_new = max(SHRINK * r_trust, R_MIN)
    return StepResult(accepted, cur, act, pred, r_new, info["kkt"], du, K, info)


def run(prob, n_steps=10, method="dr", opt=None, r0=2.0):
    u = prob.u_init.copy()
    r = r0
    K = np.zeros((prob.T, prob.nu, prob.nx))
    hist = []
    for _ in range(n_steps):
        res = step(prob, u, r, method, opt)
        if res.accepted:
            u = u + res.du.reshape(prob.T, prob.nu)
            K = res.K
        r = res.r_trust
        hist.append(res)
    return u, K, hist
