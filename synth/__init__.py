"""Seeded synthetic inputs shared by the tests, the benchmark and the CPU oracle.

This module holds random-number generation and problem *parameters* only
(start, goal, obstacles, limits, link lengths, initial guesses, random cone
vectors).  It contains none of the solver's arithmetic: no dynamics, no
linearisation, no projection, no iteration.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): state_i = seed + (i+1)*gamma,
z = mix(state_i) with the published two multiply-xorshift rounds, and a
uniform double in [0, 1) is (z >> 11) * 2**-53.  A stream is addressed by
(config, index, purpose) so every instance of every workload is reproducible
on its own.

Workloads (the robust trajectory problems of the paper's experiments section,
with the sizes used here):
  * unicycle  (n_x=3, n_u=2): Euler dt 0.1, T 20, ball radius 0.02, obstacles
    with centres U[1,4]^2 and radii U[0.3,0.6], |v|,|omega| <= 2, start
    (0,0,0), goal (5,5,0);
  * quadrotor (n_x=12, n_u=4): m 1.0, J 0.01 I, dt 0.05, T 50, ball radius
    0.05, obstacles with centres U[1,9]^3 and radii U[0.4,1.0], thrust in
    [0, 2 m g], start 0, goal position (10,10,10), hover initial guess;
  * 7-link arm (n_x=14, n_u=7): joint-space double integrator, dt 0.02, T 60,
    DH link lengths U[0.1,0.4], ball radius 0.01, 4 obstacles tested at the 7
    link frame origins, joint position and torque box bounds.
Obstacles closer than radius + 0.2 to the start or goal position are redrawn
(unicycle, quadrotor).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

DYN_UNICYCLE = 0
DYN_QUADROTOR = 1
DYN_ARM = 2

GRAVITY = 9.81

# Franka Panda joint limits and torque limits (supplementary dynamics table).
FRANKA_QMIN = np.array([-2.9007, -1.8361, -2.9007, -3.0770, -2.8763, 0.4398, -3.0508])
FRANKA_QMAX = np.array([2.9007, 1.8361, 2.9007, -0.1169, 2.8763, 4.6216, 3.0508])
FRANKA_TAUMAX = np.array([87.0, 87.0, 87.0, 87.0, 12.0, 12.0, 12.0])


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n consecutive SplitMix64 outputs of the stream that starts at `seed`."""
    with np.errstate(over="ignore"):
        idx = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def stream_seed(*keys: int) -> int:
    """Combine small integer keys into one 64-bit seed (SplitMix64 chaining)."""
    s = 0x243F6A8885A308D3
    for k in keys:
        s = int(splitmix64(s ^ (int(k) & 0xFFFFFFFFFFFFFFFF), 1)[0])
    return s


def uniform(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """n doubles uniform in [0, 1)."""
    z = splitmix64(seed, n, offset)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


class Draws:
    """Sequential consumer of one uniform stream."""

    def __init__(self, seed: int):
        self.seed = seed
        self.pos = 0

    def u(self, n: int = 1, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        v = uniform(self.seed, n, self.pos)
        self.pos += n
        return lo + (hi - lo) * v

    def ints(self, n: int, lo: int, hi: int) -> np.ndarray:
        """Integers uniform in [lo, hi] inclusive."""
        v = self.u(n)
        return lo + np.minimum((v * (hi - lo + 1)).astype(np.int64), hi - lo)


@dataclasses.dataclass
class Problem:
    """One robust trajectory problem: dynamics, horizon, cost, disturbance ball, constraints.

    Arrays are float64.  Obstacles are rows (centre..., radius).  Bounds that
    are absent are None; a bounded component has finite entries, an unbounded
    one +-inf.  For the arm, `links` holds the DH link lengths a_i.
    """
    dyn: int
    nx: int
    nu: int
    T: int
    dt: float
    radius: float                 # disturbance ball radius r = sqrt(tau)
    x0: np.ndarray
    xg: np.ndarray
    Q: np.ndarray
    Ru: np.ndarray
    RK: np.ndarray                # gain weight R_K (cost ||R_K K_k||_F^2)
    obstacles: np.ndarray         # (n_obs, d+1)
    u_lo: Optional[np.ndarray]
    u_hi: Optional[np.ndarray]
    x_lo: Optional[np.ndarray]
    x_hi: Optional[np.ndarray]
    u_init: np.ndarray            # (T, nu) initial nominal controls
    mass: float = 1.0
    inertia: Optional[np.ndarray] = None   # quadrotor diag(J)
    links: Optional[np.ndarray] = None     # arm DH link lengths (7)
    name: str = ""

    @property
    def n_obs(self) -> int:
        return int(self.obstacles.shape[0])


def _draw_obstacles(d: Draws, n: int, dim: int, lo, hi, rlo, rhi, keep_clear, margin=0.2):
    """Obstacles with centres U[lo,hi]^dim and radii U[rlo,rhi], redrawn while any
    point of `keep_clear` lies within radius + margin of the centre."""
    obs = np.zeros((n, dim + 1))
    for i in range(n):
        for _attempt in range(1000):
            c = d.u(dim, lo, hi)
            rad = float(d.u(1, rlo, rhi)[0])
            ok = all(np.linalg.norm(c - p) > rad + margin for p in keep_clear)
            if ok:
                break
        obs[i, :dim] = c
        obs[i, dim] = rad
    return obs


def unicycle(seed: int, T: int = 20, n_obs: int = 2, radius: float = 0.02) -> Problem:
    d = Draws(seed)
    x0 = np.zeros(3)
    xg = np.array([5.0, 5.0, 0.0])
    obs = _draw_obstacles(d, n_obs, 2, 1.0, 4.0, 0.3, 0.6, [x0[:2], xg[:2]])
    return Problem(dyn=DYN_UNICYCLE, nx=3, nu=2, T=T, dt=0.1, radius=radius,
                   x0=x0, xg=xg, Q=np.eye(3), Ru=0.1 * np.eye(2),
                   RK=math.sqrt(0.1) * np.eye(2), obstacles=obs,
                   u_lo=np.array([-2.0, -2.0]), u_hi=np.array([2.0, 2.0]),
                   x_lo=None, x_hi=None, u_init=np.zeros((T, 2)), name="unicycle")


def quadrotor(seed: int, T: int = 50, n_obs: int = 5, radius: float = 0.05,
              x0_pos=None, goal_pos=None) -> Problem:
    d = Draws(seed)
    m = 1.0
    x0 = np.zeros(12)
    xg = np.zeros(12)
    if x0_pos is not None:
        x0[:3] = x0_pos
    xg[:3] = goal_pos if goal_pos is not None else np.array([10.0, 10.0, 10.0])
    obs = _draw_obstacles(d, n_obs, 3, 1.0, 9.0, 0.4, 1.0, [x0[:3], xg[:3]])
    u_init = np.zeros((T, 4))
    u_init[:, 0] = m * GRAVITY
    return Problem(dyn=DYN_QUADROTOR, nx=12, nu=4, T=T, dt=0.05, radius=radius,
                   x0=x0, xg=xg, Q=np.eye(12), Ru=0.1 * np.eye(4),
                   RK=math.sqrt(0.1) * np.eye(4), obstacles=obs,
                   u_lo=np.array([0.0, -np.inf, -np.inf, -np.inf]),
                   u_hi=np.array([2 * m * GRAVITY, np.inf, np.inf, np.inf]),
                   x_lo=None, x_hi=None, u_init=u_init, mass=m,
                   inertia=np.array([0.01, 0.01, 0.01]), name="quadrotor")


def arm(seed: int, T: int = 60, n_obs: int = 4, radius: float = 0.01) -> Problem:
    """7-link DH arm as a joint-space double integrator.

    Start is the middle of the joint limits (zero lies outside the limits of
    joints 4 and 6); the goal is uniform in the middle half of each range.
    Obstacles have centres in [-0.6,0.6]^2 x [0,0.9] scaled by sum(L)/2.5 and
    radii U[0.05,0.15].  They are not tested against the start and goal poses
    (that test needs the arm's kinematics, which belong to the method).
    """
    d = Draws(seed)
    links = d.u(7, 0.1, 0.4)
    mid = 0.5 * (FRANKA_QMIN + FRANKA_QMAX)
    half = 0.5 * (FRANKA_QMAX - FRANKA_QMIN)
    q0 = mid.copy()
    qg = mid + half * d.u(7, -0.5, 0.5)
    x0 = np.concatenate([q0, np.zeros(7)])
    xg = np.concatenate([qg, np.zeros(7)])
    scale = links.sum() / 2.5
    obs = np.zeros((n_obs, 4))
    for i in range(n_obs):
        obs[i, :2] = d.u(2, -0.6, 0.6) * scale
        obs[i, 2] = d.u(1, 0.0, 0.9)[0] * scale
        obs[i, 3] = d.u(1, 0.05, 0.15)[0]
    x_lo = np.concatenate([FRANKA_QMIN, np.full(7, -np.inf)])
    x_hi = np.concatenate([FRANKA_QMAX, np.full(7, np.inf)])
    return Problem(dyn=DYN_ARM, nx=14, nu=7, T=T, dt=0.02, radius=radius,
                   x0=x0, xg=xg, Q=np.eye(14), Ru=0.1 * np.eye(7),
                   RK=math.sqrt(0.1) * np.eye(7), obstacles=obs,
                   u_lo=-FRANKA_TAUMAX.copy(), u_hi=FRANKA_TAUMAX.copy(),
                   x_lo=x_lo, x_hi=x_hi, u_init=np.zeros((T, 7)), links=links, name="arm")


# ---------------------------------------------------------------- workloads

def config1() -> Problem:
    """Unicycle, T=20, 2 obstacles, radius 0.02 (seed 1)."""
    return unicycle(stream_seed(1, 0))


def config2() -> Problem:
    """Quadrotor, T=50, 5 obstacles, radius 0.05 (seed 2)."""
    return quadrotor(stream_seed(2, 0))


def config3() -> Problem:
    """7-link arm, T=60, 4 obstacles, radius 0.01 (seed 3)."""
    return arm(stream_seed(3, 0))


def config4_instance(i: int) -> Problem:
    """Mixed batch member i of 2048: i < 1024 unicycle, else quadrotor;
    horizon U{20..80}, obstacles U{1..10}."""
    d = Draws(stream_seed(4, i, 1))
    T = int(d.ints(1, 20, 80)[0])
    n_obs = int(d.ints(1, 1, 10)[0])
    if i < 1024:
        return unicycle(stream_seed(4, i), T=T, n_obs=n_obs)
    return quadrotor(stream_seed(4, i), T=T, n_obs=n_obs)


def config5_instance(i: int, split: str = "train") -> Problem:
    """Quadrotor T=50 with 10 obstacles, start position U[0,1]^3, goal position
    U[9,10]^3.  split 'train' uses seeds (5, i), 'heldout' uses (6, i)."""
    key = 5 if split == "train" else 6
    d = Draws(stream_seed(key, i, 1))
    x0p = d.u(3, 0.0, 1.0)
    gp = d.u(3, 9.0, 10.0)
    return quadrotor(stream_seed(key, i), T=50, n_obs=10, x0_pos=x0p, goal_pos=gp)


# Sweeps shaped like the paper's unicycle / quadrotor sweep table: horizon T,
# uncertainty level tau and obstacle count varied one at a time around
# (T0, tau0, O0) = (30, 0.05, 0), step 25 ms.  The level is used as the radius of
# the disturbance ball (as the batch workloads' radii 0.02 / 0.05); goals and
# obstacles are scaled to what the systems reach in T * 25 ms.
TABLE1_NOMINAL = (30, 0.05, 0)
TABLE1_SWEEPS = {"T": (30, 45, 60), "tau": (0.025, 0.05, 0.075), "obs": (0, 3, 5)}


def table1_instance(model: str, T: int, tau: float, n_obs: int, i: int) -> Problem:
    """Instance i of one sweep point; model 'unicycle' (goal (1, 1, 0), obstacles
    with centres U[0.25, 0.75]^2 and radii U[0.04, 0.08]) or 'quadrotor' (goal
    position (1, 1, 1), centres U[0.25, 0.75]^3, radii U[0.04, 0.08]); ball
    radius tau; dt = 0.025."""
    mid = 0 if model == "unicycle" else 1
    seed = stream_seed(7, mid, T, int(round(tau * 1000)), n_obs, i)
    d = Draws(stream_seed(7, mid, i, 1))
    if model == "unicycle":
        p = unicycle(seed, T=T, n_obs=0, radius=tau)
        p.xg = np.array([1.0, 1.0, 0.0])
        p.obstacles = _draw_obstacles(d, n_obs, 2, 0.25, 0.75, 0.04, 0.08, [p.x0[:2], p.xg[:2]], margin=0.1)
    else:
        p = quadrotor(seed, T=T, n_obs=0, radius=tau, goal_pos=np.array([1.0, 1.0, 1.0]))
        p.obstacles = _draw_obstacles(d, n_obs, 3, 0.25, 0.75, 0.04, 0.08, [p.x0[:3], p.xg[:3]], margin=0.1)
    p.dt = 0.025
    p.name = f"{model} T={T} tau={tau} obs={n_obs}"
    return p


def mlp_features(p: Problem) -> np.ndarray:
    """Network input for the warm start: x0 (12), goal (12), 10 x (centre, radius)."""
    f = np.zeros(64)
    f[:12] = p.x0
    f[12:24] = p.xg
    ob = p.obstacles[:10]
    f[24:24 + ob.size] = ob.ravel()
    return f


# ------------------------------------------------------- random cone vectors

def cone_lengths(seed: int, n_cones: int, lo: int = 1, hi: int = 1024) -> np.ndarray:
    """Segment lengths for projection tests: log-uniform in [lo, hi]."""
    d = Draws(seed)
    v = d.u(n_cones)
    L = np.exp(np.log(lo) + v * (np.log(hi + 1) - np.log(lo)))
    return np.clip(L.astype(np.int64), lo, hi)


def cone_values(seed: int, n: int) -> np.ndarray:
    """Entries uniform in [-1, 1)."""
    return uniform(seed, n) * 2.0 - 1.0
