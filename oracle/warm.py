"""Learned warm start of NRTO-DR: the DR state rebuilt from a prediction of
(du, p~, pi), and the cold fallback test (test infrastructure only).

The paper names learned warm starts as future work (Conclusion); the state is
rebuilt here from the fixed-point relations of the relaxed DR splitting of the
{k_v, p~} block (supplementary II-A): with the affine-set prox's y eliminated,
the cone multiplier is zeta_j = sigma_s (eta~_j - eta_j), and a DR fixed point
has s~ = S + y / sigma_s with S = (p~, eta) the affine point and y the cone
multiplier.  The gains are those of the cold point, K = K~ = 0, so eta_j =
b_hat_j.  For a predicted (du, p~_pred, pi_pred):

  pi_j  = max(pi_pred_j, 0)
  p~_j  = max(p~_pred_j, ||eta_j||)        (the cone point (p~_j, eta_j) is feasible)
  p_j   = p~~_j = p~_j,  lambda_j = -pi_j  (p = p~ and the ADMM dual of a fixed point)
  y_j   = pi_j (1, -eta_j / ||eta_j||)     (zero eta part when eta_j = 0)
  s~_j  = (p~_j, eta_j) + y_j / sigma_s
  du    = du_pred,  mu = 0

The fallback keeps the cold point when the warm point's KKT residual (oracle.kkt)
exceeds the cold point's.
"""
from __future__ import annotations

import numpy as np

from . import dr
from .linearize import eta


def reconstruct(socp, opt: "dr.Options", du, pt_pred, pi_pred) -> "dr.State":
    st = dr.zero_state(socp)
    pi = np.maximum(np.asarray(pi_pred, dtype=np.float64), 0.0)
    E = eta(socp, st.K)                          # K = 0: eta_j = b_hat_j
    n = np.sqrt(np.sum(E * E, axis=1))
    pt = np.maximum(np.asarray(pt_pred, dtype=np.float64), n)
    st.du = np.asarray(du, dtype=np.float64).copy()
    st.p = pt.copy()
    st.pt = pt.copy()
    st.pt_t = pt.copy()
    st.pi = pi
    st.lam = -pi
    ss = opt.sigma_s
    st.s_t[:, 0] = pt + pi / ss
    safe = np.where(n > 0.0, n, 1.0)
    Y = np.where(n[:, None] > 0.0, -pi[:, None] * E / safe[:, None], 0.0)
    st.s_t[:, 1:] = E + Y / ss
    st.mu = 0.0
    st.sigma_s = ss
    return st


def warm_or_cold(socp, opt: "dr.Options", du, pt_pred, pi_pred):
    """Returns (state, accepted, residual of the warm point, residual of the cold point)."""
    cold = dr.cold_state(socp, opt)
    cold.sigma_s = opt.sigma_s
    r_cold = dr.residual(socp, opt, cold)
    warm = reconstruct(socp, opt, du, pt_pred, pi_pred)
    r_warm = dr.residual(socp, opt, warm)
    keep = r_warm <= r_cold
    return (warm if keep else cold), bool(keep), r_warm, r_cold
