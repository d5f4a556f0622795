"""Linearisation and robust constraint data (Problem 2; supplementary section I).

Everything here is dense and follows the definitions directly:

  * rollout x_{k+1} = f(x_k, u_k) from x_0 = x0 (Problem 1, nominal part);
  * linearised deviations dx = F_u du + F_zeta zeta, where zeta stacks the
    initial disturbance and d_0..d_{T-1}; block i of zeta enters x_i.  F_u and
    F_zeta are built column by column by simulating unit impulses through
    dx_{t+1} = A_t dx_t + B_t du_t + zeta_{t+1};
  * with the affine policy u_k = u_bar_k + K_k zeta_k (zeta_0 = initial
    disturbance), a constraint g_j linearised at the nominal point has the
    worst case over the ball ||zeta|| <= r equal to
        g_j^0 + b_j' du + || A_hat_j k_v + b_hat_j ||,
    b_j = F_u' grad g_j,  b_hat_j = r F_zeta' grad g_j,
    A_hat_j k_v = r [K_0' b_{j,0}; ...; K_{T-1}' b_{j,T-1}; 0]
    (supplementary section I with Gamma = S = Psi = I and sqrt(tau) = r);
  * control bounds h_j(u) = s u_{k,i} - bound have b_j = s e_{k,i}, b_hat_j = 0.

Constraint order (shared convention with the GPU library): all state
constraints first, by time t = 1..T; within one t the obstacles (for the arm:
obstacle-major, then link point 0..6), then state upper / lower bounds per
component; then control bounds by step k = 0..T-1, per input upper then lower.

The cost adds a tracking term sum_{t=1..T} (x_t - x_goal)' Q (x_t - x_goal) to
the paper's control cost (a reading: the paper's objective has no state cost).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import models

KIND_STATE = 0
KIND_CONTROL = 1


@dataclasses.dataclass
class Socp:
    nx: int
    nu: int
    T: int
    radius: float
    xhat: np.ndarray      # (T+1, nx)
    uhat: np.ndarray      # (T, nu)
    A: np.ndarray         # (T, nx, nx)
    B: np.ndarray         # (T, nx, nu)
    Fu: np.ndarray        # ((T+1)nx, T nu)
    Fz: np.ndarray        # ((T+1)nx, (T+1)nx)
    bmat: np.ndarray      # (ng, T nu)      rows b_j
    bhat: np.ndarray      # (ng, (T+1) nx)  rows b_hat_j
    g0: np.ndarray        # (ng,)
    kind: np.ndarray      # (ng,) KIND_STATE / KIND_CONTROL
    time: np.ndarray      # (ng,) t_j (state) or k_j (control)
    w: np.ndarray         # (ng, nx) gradient of a state constraint at x_{t_j}
    cidx: np.ndarray      # (ng,) input index of a control bound (-1 for state)
    csign: np.ndarray     # (ng,) +1 upper / -1 lower (0 for state)
    H: np.ndarray         # (T nu, T nu) Hessian of Q_u
    h: np.ndarray         # (T nu,) gradient of Q_u at du = 0
    c0: float             # Q_u(0)
    RK2: np.ndarray       # R_K' R_K
    Ru: np.ndarray
    Q: np.ndarray
    xg: np.ndarray
    r_trust: float

    @property
    def ng(self) -> int:
        return int(self.g0.shape[0])

    @property
    def nz(self) -> int:
        return (self.T + 1) * self.nx


def rollout(prob, u: np.ndarray) -> np.ndarray:
    x = np.zeros((prob.T + 1, prob.nx))
    x[0] = prob.x0
    for k in range(prob.T):
        x[k + 1] = models.step(prob, x[k], u[k])
    return x


def trajectory_jacobians(prob, x, u):
    A = np.zeros((prob.T, prob.nx, prob.nx))
    B = np.zeros((prob.T, prob.nx, prob.nu))
    for k in range(prob.T):
        A[k], B[k] = models.jacobians(prob, x[k], u[k])
    return A, B


def sensitivity_matrices(A, B):
    """Dense F_u and F_zeta by impulse simulation of the linearised dynamics."""
    T, nx, nu = B.shape
    Fu = np.zeros(((T + 1) * nx, T * nu))
    for k in range(T):
        for i in range(nu):
            dx = np.zeros(nx)
            for t in range(T):
                du = np.zeros(nu)
                if t == k:
                    du[i] = 1.0
                dx = A[t] @ dx + B[t] @ du
                Fu[(t + 1) * nx:(t + 2) * nx, k * nu + i] = dx
    Fz = np.zeros(((T + 1) * nx, (T + 1) * nx))
    for blk in range(T + 1):
        for i in range(nx):
            dx = np.zeros(nx)
            if blk == 0:
                dx[i] = 1.0
            Fz[0:nx, blk * nx + i] = dx
            for t in range(T):
                z = np.zeros(nx)
                if blk == t + 1:
                    z[i] = 1.0
                dx = A[t] @ dx + z
                Fz[(t + 1) * nx:(t + 2) * nx, blk * nx + i] = dx
    return Fu, Fz


def _position(prob, xt):
    """Point tested against obstacles, and its Jacobian w.r.t. the state.
    For the arm this is a list over the 7 link points."""
    if prob.dyn == 0:
        P = np.zeros((2, prob.nx))
        P[0, 0] = P[1, 1] = 1.0
        return [(xt[:2].copy(), P)]
    if prob.dyn == 1:
        P = np.zeros((3, prob.nx))
        P[0, 0] = P[1, 1] = P[2, 2] = 1.0
        return [(xt[:3].copy(), P)]
    q = xt[:7]
    pts = models.link_points(prob.links, q)
    out = []
    for i in range(7):
        Jp = np.zeros((3, prob.nx))
        Jp[:, :7] = models.link_point_jacobian(prob.links, q, i)
        out.append((pts[i], Jp))
    return out


def state_constraints_at(prob, xt):
    """(g value, gradient w.r.t. x_t) of every state constraint at one time, in canonical order."""
    out = []
    pos = _position(prob, xt)
    for o in range(prob.n_obs):
        c = prob.obstacles[o, :-1]
        rad = prob.obstacles[o, -1]
        for (pt, Jp) in pos:
            d = pt - c
            nd = float(np.linalg.norm(d))
            if nd > 0.0:
                dirv = d / nd
            else:
                dirv = np.zeros_like(d)
                dirv[0] = 1.0
            out.append((rad - nd, -(Jp.T @ dirv)))
    if prob.x_hi is not None:
        for i in range(prob.nx):
            if np.isfinite(prob.x_hi[i]):
                w = np.zeros(prob.nx)
                w[i] = 1.0
                out.append((xt[i] - prob.x_hi[i], w))
            if np.isfinite(prob.x_lo[i]):
                w = np.zeros(prob.nx)
                w[i] = -1.0
                out.append((prob.x_lo[i] - xt[i], w))
    return out


def assemble(prob, uhat: np.ndarray, r_trust: float = 2.0) -> Socp:
    """Problem 2 at the nominal controls uhat, in dense form."""
    T, nx, nu = prob.T, prob.nx, prob.nu
    xhat = rollout(prob, uhat)
    A, B = trajectory_jacobians(prob, xhat, uhat)
    Fu, Fz = sensitivity_matrices(A, B)
    r = prob.radius
    rows_b, rows_bh, g0, kind, time, W, cidx, csign = [], [], [], [], [], [], [], []
    for t in range(1, T + 1):
        for (gv, w) in state_constraints_at(prob, xhat[t]):
            grad = np.zeros((T + 1) * nx)
            grad[t * nx:(t + 1) * nx] = w
            rows_b.append(Fu.T @ grad)
            rows_bh.append(r * (Fz.T @ grad))
            g0.append(gv)
            kind.append(KIND_STATE)
            time.append(t)
            W.append(w)
            cidx.append(-1)
            csign.append(0)
    for k in range(T):
        for i in range(nu):
            for s, bound in ((1.0, None if prob.u_hi is None else prob.u_hi[i]),
                             (-1.0, None if prob.u_lo is None else prob.u_lo[i])):
                if bound is None or not np.isfinite(bound):
                    continue
                b = np.zeros(T * nu)
                b[k * nu + i] = s
                rows_b.append(b)
                rows_bh.append(np.zeros((T + 1) * nx))
                g0.append(s * uhat[k, i] - s * bound)
                kind.append(KIND_CONTROL)
                time.append(k)
                W.append(np.zeros(nx))
                cidx.append(i)
                csign.append(int(s))
    # Q_u(du) = sum_k (u+du)' Ru (u+du) + sum_{t>=1} (x+dx-xg)' Q (x+dx-xg), dx = Fu du
    Qbar = np.zeros(((T + 1) * nx, (T + 1) * nx))
    for t in range(1, T + 1):
        Qbar[t * nx:(t + 1) * nx, t * nx:(t + 1) * nx] = prob.Q
    Rbar = np.kron(np.eye(T), prob.Ru)
    dev = (xhat - prob.xg[None, :]).ravel()
    dev[:nx] = 0.0
    H = 2.0 * Rbar + 2.0 * Fu.T @ Qbar @ Fu
    h = 2.0 * Rbar @ uhat.ravel() + 2.0 * Fu.T @ Qbar @ dev
    c0 = float(uhat.ravel() @ Rbar @ uhat.ravel() + dev @ Qbar @ dev)
    return Socp(nx=nx, nu=nu, T=T, radius=r, xhat=xhat, uhat=uhat.copy(), A=A, B=B, Fu=Fu, Fz=Fz,
                bmat=np.array(rows_b), bhat=np.array(rows_bh), g0=np.array(g0),
                kind=np.array(kind, dtype=np.int32), time=np.array(time, dtype=np.int32),
                w=np.array(W), cidx=np.array(cidx, dtype=np.int32), csign=np.array(csign, dtype=np.int32),
                H=0.5 * (H + H.T), h=h, c0=c0, RK2=prob.RK.T @ prob.RK, Ru=prob.Ru.copy(),
                Q=prob.Q.copy(), xg=prob.xg.copy(), r_trust=float(r_trust))


# ----------------------------------------------------------- operators on k_v

def kv_to_K(kv: np.ndarray, T: int, nu: int, nx: int) -> np.ndarray:
    """k_v = [vec(K_0); ...] with column-major vec -> array K[k, u, x]."""
    return kv.reshape(T, nx, nu).transpose(0, 2, 1).copy()


def K_to_kv(K: np.ndarray) -> np.ndarray:
    return K.transpose(0, 2, 1).reshape(-1).copy()


def eta(socp: Socp, K: np.ndarray) -> np.ndarray:
    """Rows eta_j = A_hat_j k_v + b_hat_j, shape (ng, (T+1) nx); uses K_k' b_{j,k}."""
    T, nu, nx = socp.T, socp.nu, socp.nx
    bj = socp.bmat.reshape(-1, T, nu)
    a = np.einsum("kux,jku->jkx", K, bj)
    out = socp.bhat.copy()
    out[:, :T * nx] += socp.radius * a.reshape(-1, T * nx)
    return out


def eta_adjoint(socp: Socp, V: np.ndarray) -> np.ndarray:
    """sum_j A_hat_j' v_j as an array (T, nu, nx): block k is r sum_j b_{j,k} v_{j,k}'."""
    T, nu, nx = socp.T, socp.nu, socp.nx
    bj = socp.bmat.reshape(-1, T, nu)
    v = V[:, :T * nx].reshape(-1, T, nx)
    return socp.radius * np.einsum("jku,jkx->kux", bj, v)


def AtA_dense(socp: Socp) -> np.ndarray:
    """sum_j A_hat_j' A_hat_j in k_v coordinates: blkdiag_k(I_nx kron r^2 sum_j b_jk b_jk')."""
    T, nu, nx = socp.T, socp.nu, socp.nx
    bj = socp.bmat.reshape(-1, T, nu)
    n = T * nu * nx
    M = np.zeros((n, n))
    for k in range(T):
        G = socp.radius ** 2 * (bj[:, k, :].T @ bj[:, k, :])
        s = k * nu * nx
        M[s:s + nu * nx, s:s + nu * nx] = np.kron(np.eye(nx), G)
    return M


def Qv_dense(socp: Socp) -> np.ndarray:
    """Q_v = 2 blkdiag(I_nx kron R_K' R_K) (supplementary section I)."""
    return 2.0 * np.kron(np.eye(socp.T * socp.nx), socp.RK2)


def A_hat_dense(socp: Socp, j: int) -> np.ndarray:
    """A_hat_j written out from its definition (tests only; Gamma = S = Psi = I)."""
    T, nu, nx = socp.T, socp.nu, socp.nx
    bj = socp.bmat[j].reshape(T, nu)
    Abar = np.zeros((T * nx, T * nu * nx))
    for k in range(T):
        Abar[k * nx:(k + 1) * nx, k * nu * nx:(k + 1) * nu * nx] = np.kron(np.eye(nx), bj[k][None, :])
    return socp.radius * np.vstack([Abar, np.zeros((nx, T * nu * nx))])


def qu_value(socp: Socp, du: np.ndarray) -> float:
    return float(0.5 * du @ socp.H @ du + socp.h @ du + socp.c0)


def qk_value(socp: Socp, K: np.ndarray) -> float:
    kv = K_to_kv(K)
    return float(0.5 * kv @ Qv_dense(socp) @ kv)
