"""Seeded synthetic scenario generators for the multi-agent trajectory problem.

This module holds problem *data* only: dynamics matrices, weights, start and
goal placements, straight-line references and the ragged batch packing. It
contains none of the solver's arithmetic, so both the FP64 oracle and the HIP
path can take their inputs from it.

Problem statement followed: Sec. III-A, Eq. (1) (agents with linear dynamics,
quadratic tracking/effort cost, input box, pairwise minimum distance) and the
experimental setup of Sec. V-A (2D double integrator, n_x = 4, n_u = 2,
horizon 20, straight-line constant-velocity crossing references).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

BASE_SEED = 2602
DT = 0.1


def rng_for(config_id: int, scenario_id: int, base_seed: int = BASE_SEED) -> np.random.Generator:
    """Counter-style seeding: one independent PCG64 stream per (config, scenario)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([config_id, scenario_id, base_seed])))


def double_integrator(dp: int, dt: float = DT):
    """Exact zero-order-hold double integrator in `dp` dimensions.

    State = (position[dp], velocity[dp]); input = acceleration[dp].
    A = [[I, dt I], [0, I]], B = [[dt^2/2 I], [dt I]].
    """
    n, m = 2 * dp, dp
    A = np.eye(n)
    A[:dp, dp:] = dt * np.eye(dp)
    B = np.zeros((n, m))
    B[:dp, :] = 0.5 * dt * dt * np.eye(dp)
    B[dp:, :] = dt * np.eye(dp)
    return A, B


@dataclasses.dataclass
class ProblemParams:
    """Problem constants shared by every scenario of a batch (homogeneous agents)."""
    dp: int = 2                      # position dimension; n_x = 2 dp, n_u = dp
    dt: float = DT
    u_max: float = 2.0               # per-component box |u_c| <= u_max
    q_diag: Optional[np.ndarray] = None   # default diag(1,..,1, .1,..,.1)
    r_diag: Optional[np.ndarray] = None   # default 0.01
    qT_scale: float = 10.0           # terminal weight Q_T = qT_scale * Q
    d_min: float = 0.5
    rho: float = 1.0
    eps_abs: float = 1e-4
    eps_rel: float = 1e-4
    max_iter: int = 200

    def __post_init__(self):
        if self.q_diag is None:
            self.q_diag = np.array([1.0] * self.dp + [0.1] * self.dp)
        if self.r_diag is None:
            self.r_diag = np.full(self.dp, 0.01)
        self.q_diag = np.asarray(self.q_diag, dtype=np.float64)
        self.r_diag = np.asarray(self.r_diag, dtype=np.float64)

    @property
    def nx(self) -> int:
        return 2 * self.dp

    @property
    def nu(self) -> int:
        return self.dp

    @property
    def A(self) -> np.ndarray:
        return double_integrator(self.dp, self.dt)[0]

    @property
    def B(self) -> np.ndarray:
        return double_integrator(self.dp, self.dt)[1]

    @property
    def u_lo(self) -> np.ndarray:
        return np.full(self.nu, -self.u_max)

    @property
    def u_hi(self) -> np.ndarray:
        return np.full(self.nu, self.u_max)


@dataclasses.dataclass
class Scenario:
    """One multi-agent instance: N agents, horizon T, starts at rest, goals."""
    starts: np.ndarray   # [N][dp]
    goals: np.ndarray    # [N][dp]
    T: int
    dt: float = DT
    q_diag: Optional[np.ndarray] = None   # per-scenario override of the weights
    r_diag: Optional[np.ndarray] = None
    # heterogeneous agents: per-agent weights [N][nx], [N][nu] and input
    # boxes [N][nu] (None: the scenario's / the problem's)
    agent_q: Optional[np.ndarray] = None
    agent_r: Optional[np.ndarray] = None
    agent_lo: Optional[np.ndarray] = None
    agent_hi: Optional[np.ndarray] = None
    # per-agent dynamics [N][nx][nx], [N][nx][nu] (None: the problem's)
    agent_A: Optional[np.ndarray] = None
    agent_B: Optional[np.ndarray] = None

    @property
    def N(self) -> int:
        return int(self.starts.shape[0])

    @property
    def dp(self) -> int:
        return int(self.starts.shape[1])

    @property
    def P(self) -> int:
        return self.N * (self.N - 1) // 2

    def x0(self) -> np.ndarray:
        """Initial states: start positions, zero velocity.  [N][nx]"""
        return np.concatenate([self.starts, np.zeros_like(self.starts)], axis=1)

    def xref(self) -> np.ndarray:
        """Straight-line constant-velocity references, t = 0..T.  [N][T+1][nx]

        r_t = (p_s + (t/T)(g - p_s), (g - p_s)/(T dt)) (Sec. V-A: straight lines
        with constant velocity that make the agents cross).
        """
        return straight_line_ref(self.starts, self.goals, self.T, self.dt)


def straight_line_ref(starts: np.ndarray, goals: np.ndarray, T: int, dt: float = DT) -> np.ndarray:
    starts = np.asarray(starts, dtype=np.float64)
    goals = np.asarray(goals, dtype=np.float64)
    N, dp = starts.shape
    frac = np.arange(T + 1, dtype=np.float64) / T                  # [T+1]
    pos = starts[:, None, :] + frac[None, :, None] * (goals - starts)[:, None, :]
    vel = np.broadcast_to(((goals - starts) / (T * dt))[:, None, :], (N, T + 1, dp))
    return np.concatenate([pos, vel], axis=2)


# ----------------------------------------------------------------------------
# Workload generators
# ----------------------------------------------------------------------------

def circle_swap(N: int, radius: float, T: int, jitter: float, rng: Optional[np.random.Generator],
                dt: float = DT) -> Scenario:
    """N agents evenly spaced on a circle, each heading to its antipode.

    The start positions get independent N(0, jitter^2) noise per coordinate;
    the goals are the nominal (unjittered) antipodes.
    """
    ang = 2.0 * math.pi * np.arange(N) / N
    nominal = radius * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    starts = nominal.copy()
    if jitter > 0:
        starts = starts + rng.normal(0.0, jitter, size=starts.shape)
    goals = -nominal
    return Scenario(starts=starts, goals=goals, T=T, dt=dt)


def fibonacci_sphere(N: int, radius: float) -> np.ndarray:
    """Golden-angle spiral points on a sphere.  [N][3]"""
    i = np.arange(N, dtype=np.float64)
    y = 1.0 - 2.0 * (i + 0.5) / N
    r = np.sqrt(np.maximum(0.0, 1.0 - y * y))
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    return radius * np.stack([r * np.cos(phi), y, r * np.sin(phi)], axis=1)


def sphere_swap(N: int, radius: float, T: int, dt: float = DT) -> Scenario:
    pts = fibonacci_sphere(N, radius)
    return Scenario(starts=pts, goals=-pts, T=T, dt=dt)


def _rejection_points(rng: np.random.Generator, n: int, lo: float, hi: float, min_sep: float,
                      dp: int = 2) -> np.ndarray:
    """Sequential rejection sampling: redraw each point until it is at least
    `min_sep` from every earlier point."""
    pts = np.zeros((n, dp))
    for k in range(n):
        for _ in range(100000):
            c = rng.uniform(lo, hi, size=dp)
            if k == 0 or np.min(np.linalg.norm(pts[:k] - c, axis=1)) >= min_sep:
                pts[k] = c
                break
        else:  # pragma: no cover - never reached at the sizes used
            raise RuntimeError("rejection sampling did not place a point")
    return pts


def random_box(rng: np.random.Generator, N: int, T: int, half: float = 5.0, min_sep: float = 1.0,
               dt: float = DT, dp: int = 2) -> Scenario:
    starts = _rejection_points(rng, N, -half, half, min_sep, dp)
    goals = _rejection_points(rng, N, -half, half, min_sep, dp)
    return Scenario(starts=starts, goals=goals, T=T, dt=dt)


# The five workloads.  Each returns (ProblemParams, [Scenario]).

def config0(seed_offset: int = 0):
    """2 agents, 2D double integrator, T = 20, antipodes on a radius-3 circle."""
    p = ProblemParams(dp=2, u_max=2.0)
    sc = circle_swap(2, 3.0, 20, 0.05, rng_for(0, seed_offset))
    return p, [sc]


def config1(seed_offset: int = 0, jitter: float = 0.05):
    """14 agents on a radius-4 circle swapping to antipodes, T = 20."""
    p = ProblemParams(dp=2, u_max=2.0)
    sc = circle_swap(14, 4.0, 20, jitter, rng_for(1, seed_offset))
    return p, [sc]


def config2_dims(S: int = 4096):
    """Agent counts and horizons of the ragged batch (N ~ U{2..32}, T ~ U{10..40})."""
    Ns, Ts = [], []
    for s in range(S):
        rng = rng_for(2, s)
        Ns.append(int(rng.integers(2, 33)))
        Ts.append(int(rng.integers(10, 41)))
    return Ns, Ts


def config2(S: int = 4096, scenario_ids: Optional[Sequence[int]] = None):
    """Ragged batch: N ~ U{2..32}, T ~ U{10..40}, starts/goals ~ U([-5,5]^2)
    with sequential rejection to >= 1.0 separation."""
    p = ProblemParams(dp=2, u_max=2.0)
    ids = range(S) if scenario_ids is None else scenario_ids
    out = []
    for s in ids:
        rng = rng_for(2, s)
        N = int(rng.integers(2, 33))
        T = int(rng.integers(10, 41))
        out.append(random_box(rng, N, T))
    return p, out


def config3(S: int = 256, scenario_ids: Optional[Sequence[int]] = None):
    """Differentiation batch: S scenarios of 8 agents, T = 20, random box."""
    p = ProblemParams(dp=2, u_max=2.0)
    ids = range(S) if scenario_ids is None else scenario_ids
    return p, [random_box(rng_for(3, s), 8, 20) for s in ids]


def config4():
    """128 agents, 3D double integrator, T = 50, Fibonacci sphere of radius 12,
    |u_c| <= 3."""
    p = ProblemParams(dp=3, u_max=3.0)
    return p, [sphere_swap(128, 12.0, 50)]


# ----------------------------------------------------------------------------
# Ragged packing
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class PackedBatch:
    """Flat arrays of a ragged batch.

    Ordering (all arrays are row-major, scenarios back to back):
      x0     [sum N_s][nx]              (scenario, agent)
      xref   [sum N_s (T_s+1)][nx]      (scenario, agent, t)
      q_diag [S][nx], r_diag [S][nu]
    """
    n_agents: np.ndarray    # int32 [S]
    horizon: np.ndarray     # int32 [S]
    x0: np.ndarray
    xref: np.ndarray
    q_diag: np.ndarray
    r_diag: np.ndarray
    agent_q: Optional[np.ndarray] = None    # [sum N_s][nx] (heterogeneous agents)
    agent_r: Optional[np.ndarray] = None    # [sum N_s][nu]
    agent_lo: Optional[np.ndarray] = None   # [sum N_s][nu]
    agent_hi: Optional[np.ndarray] = None   # [sum N_s][nu]
    agent_A: Optional[np.ndarray] = None    # [sum N_s][nx*nx] (per-agent dynamics)
    agent_B: Optional[np.ndarray] = None    # [sum N_s][nx*nu]

    @property
    def S(self) -> int:
        return int(self.n_agents.shape[0])

    def agent_off(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.n_agents)]).astype(np.int64)

    def traj_off(self) -> np.ndarray:
        """Offsets of scenario blocks in units of agent-stages (N_s (T_s+1))."""
        return np.concatenate([[0], np.cumsum(self.n_agents * (self.horizon + 1))]).astype(np.int64)

    def input_off(self) -> np.ndarray:
        """Offsets in units of agent-input-stages (N_s T_s)."""
        return np.concatenate([[0], np.cumsum(self.n_agents * self.horizon)]).astype(np.int64)

    def pair_step_off(self) -> np.ndarray:
        """Offsets in units of pair-steps (P_s T_s), P_s = N_s (N_s - 1) / 2."""
        P = self.n_agents * (self.n_agents - 1) // 2
        return np.concatenate([[0], np.cumsum(P * self.horizon)]).astype(np.int64)


def pack(params: ProblemParams, scenarios: List[Scenario], dtype=np.float64) -> PackedBatch:
    nx, nu = params.nx, params.nu
    Ns = np.array([sc.N for sc in scenarios], dtype=np.int32)
    Ts = np.array([sc.T for sc in scenarios], dtype=np.int32)
    x0 = np.concatenate([sc.x0() for sc in scenarios], axis=0).astype(dtype) if scenarios else np.zeros((0, nx), dtype)
    xref = (np.concatenate([sc.xref().reshape(-1, nx) for sc in scenarios], axis=0).astype(dtype)
            if scenarios else np.zeros((0, nx), dtype))
    q = np.stack([(params.q_diag if sc.q_diag is None else sc.q_diag) for sc in scenarios]).astype(dtype) \
        if scenarios else np.zeros((0, nx), dtype)
    r = np.stack([(params.r_diag if sc.r_diag is None else sc.r_diag) for sc in scenarios]).astype(dtype) \
        if scenarios else np.zeros((0, nu), dtype)
    pb = PackedBatch(Ns, Ts, x0, xref, q, r)
    if any(getattr(sc, f) is not None for sc in scenarios for f in ("agent_q", "agent_r", "agent_lo", "agent_hi")):
        # every agent's own values, the scenario's / problem's where not given
        def per_agent(field, fallback, width):
            return np.concatenate([np.asarray(getattr(sc, field), np.float64).reshape(sc.N, width)
                                   if getattr(sc, field) is not None else
                                   np.tile(np.asarray(fallback(sc), np.float64), (sc.N, 1))
                                   for sc in scenarios]).astype(dtype)
        pb.agent_q = per_agent("agent_q", lambda sc: params.q_diag if sc.q_diag is None else sc.q_diag, nx)
        pb.agent_r = per_agent("agent_r", lambda sc: params.r_diag if sc.r_diag is None else sc.r_diag, nu)
        pb.agent_lo = per_agent("agent_lo", lambda sc: params.u_lo, nu)
        pb.agent_hi = per_agent("agent_hi", lambda sc: params.u_hi, nu)
    if any(getattr(sc, f) is not None for sc in scenarios for f in ("agent_A", "agent_B")):
        def per_agent_dyn(field, fallback, width):
            return np.concatenate([np.asarray(getattr(sc, field), np.float64).reshape(sc.N, width)
                                   if getattr(sc, field) is not None else
                                   np.tile(np.asarray(fallback, np.float64).reshape(1, width), (sc.N, 1))
                                   for sc in scenarios]).astype(dtype)
        pb.agent_A = per_agent_dyn("agent_A", params.A, nx * nx)
        pb.agent_B = per_agent_dyn("agent_B", params.B, nx * nu)
    return pb


def heterogeneous(rng: np.random.Generator, sc: Scenario, params: ProblemParams, spread: float = 4.0) -> Scenario:
    """The same scenario with heterogeneous agents: each agent's Q and R
    diagonals scaled by log-uniform factors in [1/spread, spread], and its
    input box |u_c| <= u_max * U(0.5, 1.5) per component."""
    N, nx, nu = sc.N, params.nx, params.nu
    f = lambda shape: np.exp(rng.uniform(-np.log(spread), np.log(spread), size=shape))
    q = (params.q_diag if sc.q_diag is None else sc.q_diag)[None, :] * f((N, nx))
    r = (params.r_diag if sc.r_diag is None else sc.r_diag)[None, :] * f((N, nu))
    umax = params.u_max * rng.uniform(0.5, 1.5, size=(N, nu))
    return dataclasses.replace(sc, agent_q=q, agent_r=r, agent_lo=-umax, agent_hi=umax)


def damped_point_mass(dp: int, dt: float, drag: float, mass: float):
    """Exact zero-order-hold discretization of p' = v, v' = -drag v + u / mass
    in `dp` dimensions (positions first), by the matrix exponential of the
    augmented continuous system [[Ac, Bc], [0, 0]] dt."""
    import scipy.linalg
    n, m = 2 * dp, dp
    M = np.zeros((n + m, n + m))
    M[:dp, dp:n] = np.eye(dp)
    M[dp:n, dp:n] = -drag * np.eye(dp)
    M[dp:n, n:] = np.eye(dp) / mass
    E = scipy.linalg.expm(M * dt)
    return E[:n, :n], E[:n, n:]


def mixed_dynamics(rng: np.random.Generator, sc: Scenario, params: ProblemParams, drag=(0.0, 1.5),
                   mass=(0.5, 2.0)) -> Scenario:
    """The same scenario with per-agent dynamics: each agent a damped point
    mass with drag ~ U(drag) and mass ~ U(mass), exactly discretized."""
    As, Bs = [], []
    for _ in range(sc.N):
        A, B = damped_point_mass(params.dp, sc.dt, rng.uniform(*drag), rng.uniform(*mass))
        As.append(A)
        Bs.append(B)
    return dataclasses.replace(sc, agent_A=np.stack(As), agent_B=np.stack(Bs))


def problem_dimensions(N: int, T: int, nx: int = 4, nu: int = 2):
    """Problem size of the centralized QP (Eq. 1 / compact form Eq. 6).

    Returns (variables, dynamics rows, collision rows): variables count the
    stacked x_i in R^{(T+1) n} and u_i in R^{T m} of every agent; dynamics rows
    are T n per agent; collision rows count every pair at the T+1 knots.
    """
    P = N * (N - 1) // 2
    return N * ((T + 1) * nx + T * nu), N * T * nx, P * (T + 1)
