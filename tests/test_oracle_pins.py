"""Pins of the FP64 oracle against things other than itself.

Each test names what fixes the expected value: a printed table of the paper,
a closed form, a library routine solving the same problem by another method,
brute force on a tiny instance, a KKT certificate, or an invariance of the
problem.  None of them re-types the oracle's own formulas.
"""
import copy
import math
import os

import dataclasses

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize

import oracle
import synth
from tests import condensed

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Table I (Sec. V-A): problem dimensions of the centralized QP
# ---------------------------------------------------------------------------

def test_table1_problem_dimensions():
    rows = [list(map(int, l.split())) for l in open(os.path.join(GOLDEN, "table1_problem_dimensions.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for N, nvar, ndyn, ncol in rows:
        v, d, c = synth.problem_dimensions(N, 20)
        assert v == nvar and d == ndyn
        # the table prints the collision count with "~"; 2 agents: 1 pair x 21 knots printed as ~20
        assert abs(c - ncol) <= 1


# ---------------------------------------------------------------------------
# One agent's local QP (Eq. 3)
# ---------------------------------------------------------------------------

def _wide(dp=2):
    return synth.ProblemParams(dp=dp, u_max=1e6)


@pytest.mark.parametrize("dp", [2, 3])
def test_agent_qp_unconstrained_matches_condensed_least_squares(dp):
    """Pins the KKT assembly (factors of 2, terminal weight at T, the sign of
    the consensus term) against the state-eliminated least-squares form."""
    rng = np.random.default_rng(11)
    p = _wide(dp)
    T, n_nbr, rho = 12, 3, 1.7
    x0 = rng.normal(size=p.nx)
    xref = rng.normal(size=(T + 1, p.nx))
    z = rng.normal(size=(n_nbr, T + 1, dp))
    lam = rng.normal(size=(n_nbr, T + 1, dp))
    ysum = (rho * z - lam).sum(axis=0)
    q = rng.uniform(0.2, 2.0, size=p.nx)
    r = rng.uniform(0.01, 0.5, size=p.nu)
    res = oracle.agent_qp(p, T, n_nbr, x0, xref, q, r, ysum, opts=oracle.OracleOptions(rho=rho))
    J, b = condensed.agent_ls(p.A, p.B, T, x0, xref, q, r, p.qT_scale, rho, z, lam)
    u_ls = np.linalg.lstsq(J, b, rcond=None)[0].reshape(T, p.nu)
    np.testing.assert_allclose(res["u"], u_ls, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(res["x"], condensed.rollout(p.A, p.B, x0, u_ls), rtol=1e-9, atol=1e-10)
    assert not res["w"].any()


def test_agent_qp_long_horizon_first_gain_is_dare():
    """Infinite-horizon limit: with zero reference and no coupling the first
    input tends to -K x0, K from the discrete algebraic Riccati equation."""
    p = _wide(2)
    T = 200
    Q, R = np.diag(p.q_diag), np.diag(p.r_diag)
    P = scipy.linalg.solve_discrete_are(p.A, p.B, Q, R)
    K = np.linalg.solve(R + p.B.T @ P @ p.B, p.B.T @ P @ p.A)
    x0 = np.array([1.0, -2.0, 0.3, 0.5])
    res = oracle.agent_qp(p, T, 0, x0, np.zeros((T + 1, 4)), p.q_diag, p.r_diag)
    np.testing.assert_allclose(res["u"][0], -K @ x0, rtol=1e-8, atol=1e-10)


def _bounded_case(seed, T, u_max=0.6, dp=2):
    rng = np.random.default_rng(seed)
    p = synth.ProblemParams(dp=dp, u_max=u_max)
    n_nbr, rho = 2, 1.0
    x0 = np.concatenate([rng.normal(size=dp), rng.normal(scale=0.3, size=dp)])
    sc = synth.Scenario(starts=x0[None, :dp], goals=x0[None, :dp] + rng.uniform(2, 4, size=(1, dp)), T=T)
    xref = sc.xref()[0]
    z = xref[None, :, :dp] + rng.normal(scale=0.3, size=(n_nbr, T + 1, dp))
    lam = rng.normal(scale=0.5, size=(n_nbr, T + 1, dp))
    ysum = (rho * z - lam).sum(axis=0)
    return p, n_nbr, rho, x0, xref, z, lam, ysum


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_agent_qp_bounded_matches_bvls(seed):
    """Input-box QP against scipy's bounded-variable least squares (an exact
    active-set method on the condensed form): same inputs, same binding set,
    and multipliers equal to the signed gradient of the condensed objective."""
    T = 15
    p, n_nbr, rho, x0, xref, z, lam, ysum = _bounded_case(seed, T)
    res = oracle.agent_qp(p, T, n_nbr, x0, xref, p.q_diag, p.r_diag, ysum)
    J, b = condensed.agent_ls(p.A, p.B, T, x0, xref, p.q_diag, p.r_diag, p.qT_scale, rho, z, lam)
    lo, hi = np.full(T * p.nu, -p.u_max), np.full(T * p.nu, p.u_max)
    ls = scipy.optimize.lsq_linear(J, b, bounds=(lo, hi), method="bvls", tol=1e-14)
    np.testing.assert_allclose(res["u"].ravel(), ls.x, atol=1e-8)
    g = 2.0 * J.T @ (J @ res["u"].ravel() - b)
    Wf = res["w"].ravel()
    assert Wf.any(), "case should have binding bounds"
    np.testing.assert_array_equal(Wf == 1, np.isclose(ls.x, lo, atol=1e-9) & (g > 1e-7))
    np.testing.assert_array_equal(Wf == 2, np.isclose(ls.x, hi, atol=1e-9) & (g < -1e-7))
    mu = res["mu"].ravel()
    np.testing.assert_allclose(mu[Wf == 1], g[Wf == 1], rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(mu[Wf == 2], -g[Wf == 2], rtol=1e-7, atol=1e-9)
    assert np.all(mu >= -1e-9)
    np.testing.assert_allclose(g[Wf == 0], 0.0, atol=1e-8)


@pytest.mark.parametrize("seed,T", [(5, 2), (6, 3), (7, 3)])
def test_agent_qp_tiny_horizon_brute_force(seed, T):
    """T <= 3: every free/lower/upper pattern of the T*nu inputs is tried;
    exactly one is a KKT point and it is the oracle's solution."""
    p, n_nbr, rho, x0, xref, z, lam, ysum = _bounded_case(seed, T, u_max=0.8)
    J, b = condensed.agent_ls(p.A, p.B, T, x0, xref, p.q_diag, p.r_diag, p.qT_scale, rho, z, lam)
    lo, hi = np.full(T * p.nu, -p.u_max), np.full(T * p.nu, p.u_max)
    kkt = condensed.enumerate_active_sets(J, b, lo, hi)
    assert len(kkt) == 1
    pat, u = kkt[0]
    res = oracle.agent_qp(p, T, n_nbr, x0, xref, p.q_diag, p.r_diag, ysum)
    np.testing.assert_allclose(res["u"].ravel(), u, atol=1e-10)
    np.testing.assert_array_equal(res["w"].ravel(), pat)


@pytest.mark.parametrize("start", [oracle.START_WARM, oracle.START_COLD])
def test_agent_qp_start_does_not_change_the_optimum(start):
    """Warm (unconstrained solve + clip) and cold (u = 0) starts reach the
    same unique optimum; the warm start needs no more equality solves."""
    T = 20
    p, n_nbr, rho, x0, xref, z, lam, ysum = _bounded_case(9, T, u_max=0.5)
    ref = oracle.agent_qp(p, T, n_nbr, x0, xref, p.q_diag, p.r_diag, ysum, start=oracle.START_WARM)
    res = oracle.agent_qp(p, T, n_nbr, x0, xref, p.q_diag, p.r_diag, ysum, start=start)
    np.testing.assert_allclose(res["u"], ref["u"], atol=1e-10)
    np.testing.assert_array_equal(res["w"], ref["w"])
    cold = oracle.agent_qp(p, T, n_nbr, x0, xref, p.q_diag, p.r_diag, ysum, start=oracle.START_COLD)
    assert ref["passes"] <= cold["passes"]


def test_agent_qp_dynamics_and_box_feasible():
    T = 25
    p, n_nbr, rho, x0, xref, z, lam, ysum = _bounded_case(4, T, u_max=0.4)
    res = oracle.agent_qp(p, T, n_nbr, x0, xref, p.q_diag, p.r_diag, ysum)
    x, u = res["x"], res["u"]
    np.testing.assert_allclose(x[0], x0, atol=0)
    dyn = x[1:] - (x[:-1] @ p.A.T + u @ p.B.T)
    assert np.abs(dyn).max() < 1e-12
    assert np.all(u >= -p.u_max - 1e-15) and np.all(u <= p.u_max + 1e-15)
    np.testing.assert_array_equal(u[res["w"] == 1], -p.u_max)
    np.testing.assert_array_equal(u[res["w"] == 2], p.u_max)


def test_agent_qp_hotstart_from_previous_solution():
    """Starting from the optimum of a nearby QP with its working set gives the
    new optimum (the parametric hotstart of Sec. IV-C)."""
    T = 20
    p, n_nbr, rho, x0, xref, z, lam, ysum = _bounded_case(12, T, u_max=0.5)
    a = oracle.agent_qp(p, T, n_nbr, x0, xref, p.q_diag, p.r_diag, ysum)
    ysum2 = ysum + 0.05 * np.random.default_rng(1).normal(size=ysum.shape)
    cold = oracle.agent_qp(p, T, n_nbr, x0, xref, p.q_diag, p.r_diag, ysum2)
    hot = oracle.agent_qp(p, T, n_nbr, x0, xref, p.q_diag, p.r_diag, ysum2, start=oracle.START_PREV,
                          x=a["x"], u=a["u"], w=a["w"])
    np.testing.assert_allclose(hot["u"], cold["u"], atol=1e-10)
    np.testing.assert_array_equal(hot["w"], cold["w"])


def test_agent_qp_active_set_cap():
    T = 20
    p, n_nbr, rho, x0, xref, z, lam, ysum = _bounded_case(3, T, u_max=0.2)
    res = oracle.agent_qp(p, T, n_nbr, x0, xref, p.q_diag, p.r_diag, ysum,
                          start=oracle.START_COLD, opts=oracle.OracleOptions(max_as_iter=1))
    assert res["capped"]


# ---------------------------------------------------------------------------
# ADMM (Eqs. 3-5): the limit with frozen normals is the centralized QP
# ---------------------------------------------------------------------------

def _side_pass(T=20):
    """Two agents passing side by side; point-symmetric about the origin."""
    sc = synth.Scenario(starts=np.array([[-3.0, 0.6], [3.0, -0.6]]),
                        goals=np.array([[3.0, 0.1], [-3.0, -0.1]]), T=T)
    nrm = np.zeros((1, T, 2))
    nrm[..., 1] = 1.0
    return sc, nrm


def _monolithic_pieces(p, sc, normals):
    """Condensed centralized QP of Eq. (1) with the half-planes of Sec. III-A:
    f(U) = sum_i ||J_i u_i - b_i||^2, G U >= h, lo <= U <= hi."""
    N, T, nu, dp = sc.N, sc.T, p.nu, p.dp
    Phi, Gam = condensed.state_maps(p.A, p.B, T)
    Js, bs = [], []
    x0 = sc.x0()
    xref = sc.xref()
    for i in range(N):
        J, b = condensed.agent_ls(p.A, p.B, T, x0[i], xref[i], p.q_diag, p.r_diag, p.qT_scale)
        Js.append(J)
        bs.append(b)
    J = scipy.linalg.block_diag(*Js)
    b = np.concatenate(bs)
    n = T * nu
    G, h = [], []
    pidx = 0
    for i in range(N):
        for j in range(i + 1, N):
            for t in range(1, T + 1):
                nv = normals[pidx, t - 1]
                row = np.zeros(N * n)
                row[i * n:(i + 1) * n] = nv @ Gam[t][:dp]
                row[j * n:(j + 1) * n] = -nv @ Gam[t][:dp]
                G.append(row)
                h.append(p.d_min - nv @ ((Phi[t] @ x0[i])[:dp] - (Phi[t] @ x0[j])[:dp]))
            pidx += 1
    return J, b, np.array(G), np.array(h)


def test_admm_frozen_limit_is_centralized_qp_kkt_certificate():
    """C.1: with fixed normals the ADMM fixed point solves the strictly convex
    centralized QP.  Certificate: primal feasibility plus nonnegative
    multipliers on the binding bounds and half-planes that make the gradient of
    the centralized objective vanish (solved here by least squares)."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc, nrm = _side_pass()
    res = oracle.solve(p, sc, oracle.OracleOptions(normal_mode=oracle.NORMAL_FROZEN, rho=10.0, max_iter=5000,
                                                   eps_abs=1e-11, eps_rel=1e-11), normals=nrm)
    assert res["status"] == oracle.CONVERGED
    J, b, G, h = _monolithic_pieces(p, sc, nrm)
    U = res["u"].reshape(-1)
    assert np.all(G @ U - h >= -1e-7)
    grad = 2.0 * J.T @ (J @ U - b)
    W = res["w"].reshape(-1)
    cols, signs = [], []
    for k in np.nonzero(W)[0]:
        e = np.zeros(U.size)
        e[k] = 1.0 if W[k] == 1 else -1.0     # gradient of the binding constraint (>= form)
        cols.append(e)
    act = np.nonzero(np.abs(G @ U - h) < 1e-6)[0]
    assert act.size >= 1, "the half-plane should bind in this case"
    for k in act:
        cols.append(G[k])
    M = np.array(cols).T
    m, *_ = np.linalg.lstsq(M, grad, rcond=None)
    assert np.linalg.norm(M @ m - grad) < 1e-6 * (1 + np.linalg.norm(grad))
    assert np.all(m >= -1e-7)


def test_admm_adaptive_rho_frozen_limit_is_the_same_kkt_point():
    """Residual balancing (Boyd et al. 2011, Sec. 3.4.1) changes the path,
    not the fixed point: from a penalty 100x too large the run adapts rho,
    and its limit passes the same centralized-QP certificate and equals the
    fixed-penalty limit."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc, nrm = _side_pass()
    tight = dict(normal_mode=oracle.NORMAL_FROZEN, max_iter=20000, eps_abs=1e-11, eps_rel=1e-11)
    res = oracle.solve(p, sc, oracle.OracleOptions(rho=1000.0, adaptive_rho=True, **tight), normals=nrm)
    assert res["status"] == oracle.CONVERGED
    assert len(np.unique(res["rho_hist"])) >= 3 and res["rho_hist"][-1] < 1000.0
    fixed = oracle.solve(p, sc, oracle.OracleOptions(rho=10.0, **tight), normals=nrm)
    np.testing.assert_allclose(res["u"], fixed["u"], atol=1e-7)
    J, b, G, h = _monolithic_pieces(p, sc, nrm)
    U = res["u"].reshape(-1)
    assert np.all(G @ U - h >= -1e-7)
    grad = 2.0 * J.T @ (J @ U - b)
    W = res["w"].reshape(-1)
    cols = []
    for k in np.nonzero(W)[0]:
        e = np.zeros(U.size)
        e[k] = 1.0 if W[k] == 1 else -1.0
        cols.append(e)
    for k in np.nonzero(np.abs(G @ U - h) < 1e-6)[0]:
        cols.append(G[k])
    M = np.array(cols).T
    m, *_ = np.linalg.lstsq(M, grad, rcond=None)
    assert np.linalg.norm(M @ m - grad) < 1e-6 * (1 + np.linalg.norm(grad))
    assert np.all(m >= -1e-7)


def _box_certificate(p, sc, nrm, res, k0, lo, hi, what):
    """Centralized-QP certificate with state rows x_t[k0 + c] = (Phi_t x0 +
    Gam_t u)[k0 + c] in [lo_c, hi_c] (t = 1..T) among the constraints: the
    solution is feasible, the box binds, and the objective's gradient is a
    nonnegative combination of the binding rows (nonnegative least squares:
    the active rows can be dependent, e.g. a bound input and the state rows
    it drives)."""
    T, dp = sc.T, p.dp
    J, b, G, h = _monolithic_pieces(p, sc, nrm)
    Phi, Gam = condensed.state_maps(p.A, p.B, T)
    n = T * p.nu
    x0 = sc.x0()
    rows, rhs = [], []
    for i in range(sc.N):
        for t in range(1, T + 1):
            for c in range(dp):
                g = np.zeros(sc.N * n)
                g[i * n:(i + 1) * n] = Gam[t][k0 + c]
                s0 = (Phi[t] @ x0[i])[k0 + c]
                rows += [g, -g]
                rhs += [lo[c] - s0, -(hi[c] - s0)]
    G = np.vstack([G, np.array(rows)])
    h = np.concatenate([h, np.array(rhs)])
    U = res["u"].reshape(-1)
    slack = G @ U - h
    assert np.all(slack >= -1e-7)
    nbox = len(rows)
    assert np.sum(np.abs(slack[-nbox:]) < 1e-6) >= 1, f"the {what} box should bind"
    grad = 2.0 * J.T @ (J @ U - b)
    W = res["w"].reshape(-1)
    cols = []
    for k in np.nonzero(W)[0]:
        e = np.zeros(U.size)
        e[k] = 1.0 if W[k] == 1 else -1.0
        cols.append(e)
    for k in np.nonzero(np.abs(slack) < 1e-6)[0]:
        cols.append(G[k])
    M = np.array(cols).T
    m, resid = scipy.optimize.nnls(M, grad)
    assert resid < 1e-6 * (1 + np.linalg.norm(grad))


def test_admm_state_box_frozen_limit_is_centralized_qp_kkt_certificate():
    """The state box (a further ADMM split on the velocities): with fixed
    normals the limit solves the centralized QP with the velocity box added
    (certificate above, with the velocity rows v_t in [-vmax, vmax])."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc, nrm = _side_pass()
    vmax = 2.5    # off the grid of multiples of u_max dt (degenerate there)
    res = oracle.solve(p, sc, oracle.OracleOptions(normal_mode=oracle.NORMAL_FROZEN, rho=10.0, max_iter=3000,
                                                   eps_abs=1e-11, eps_rel=1e-11, state_box=True,
                                                   s_lo=(-vmax,) * 3, s_hi=(vmax,) * 3), normals=nrm)
    assert res["status"] == oracle.CONVERGED
    _box_certificate(p, sc, nrm, res, p.dp, (-vmax,) * 2, (vmax,) * 2, "velocity")


def _box_pass(T=30):
    """Two agents passing side by side towards goals beyond x = +-3."""
    sc = synth.Scenario(starts=np.array([[-2.0, 0.6], [2.0, -0.6]]),
                        goals=np.array([[3.5, 0.1], [-3.5, -0.1]]), T=T)
    nrm = np.zeros((1, T, 2))
    nrm[..., 1] = 1.0
    return sc, nrm


def test_admm_position_box_frozen_limit_is_centralized_qp_kkt_certificate():
    """The position box (the same split on the positions, whose rows then
    carry both the consensus and the box penalty): the limit solves the
    centralized QP with the position rows p_t in [-3, 3] x [-1, 1]; the
    x bound binds (the goals lie beyond it)."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc, nrm = _box_pass()
    lo, hi = (-3.0, -1.0), (3.0, 1.0)
    res = oracle.solve(p, sc, oracle.OracleOptions(normal_mode=oracle.NORMAL_FROZEN, rho=10.0, max_iter=3000,
                                                   eps_abs=1e-11, eps_rel=1e-11, state_box=True,
                                                   p_lo=lo + (0.0,), p_hi=hi + (0.0,)), normals=nrm)
    assert res["status"] == oracle.CONVERGED
    _box_certificate(p, sc, nrm, res, 0, lo, hi, "position")


def test_admm_position_box_with_adaptive_rho_same_certified_limit():
    """Residual balancing keeps the box's sigma (the initial penalty) on the
    position rows while rho moves (here from 3 up to 24 and down to 1.5):
    the adaptive run's limit passes the same certificate.  A shorter pass
    (T = 20, |x| <= 2.2) keeps the pin fast."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    T = 20
    sc = synth.Scenario(starts=np.array([[-1.5, 0.6], [1.5, -0.6]]), goals=np.array([[3.5, 0.1], [-3.5, -0.1]]), T=T)
    nrm = np.zeros((1, T, 2))
    nrm[..., 1] = 1.0
    lo, hi = (-2.2, -1.0), (2.2, 1.0)
    res = oracle.solve(p, sc, oracle.OracleOptions(normal_mode=oracle.NORMAL_FROZEN, rho=3.0, adaptive_rho=True,
                                                   rho_mu=5.0, max_iter=1000, eps_abs=1e-11, eps_rel=1e-11,
                                                   state_box=True, p_lo=lo + (0.0,), p_hi=hi + (0.0,)), normals=nrm)
    assert res["status"] == oracle.CONVERGED and len(np.unique(res["rho_hist"][:res["iters"]])) >= 3
    _box_certificate(p, sc, nrm, res, 0, lo, hi, "position")


def test_admm_state_box_groups_split_only_where_bounded():
    """A group of states with no finite bound is not split: infinite bounds
    reproduce the unboxed run bitwise, and a velocity box leaves the
    iterates of an infinite position box unchanged."""
    p, scs = synth.config2(S=3)
    sc = scs[2]
    base = dict(max_iter=30, fixed_iters=30)
    plain = oracle.solve(p, sc, oracle.OracleOptions(**base))
    inf = oracle.solve(p, sc, oracle.OracleOptions(state_box=True, **base))
    np.testing.assert_array_equal(plain["x"], inf["x"])
    vel = oracle.solve(p, sc, oracle.OracleOptions(state_box=True, s_lo=(-2.0,) * 3, s_hi=(2.0,) * 3, **base))
    both = oracle.solve(p, sc, oracle.OracleOptions(state_box=True, s_lo=(-2.0,) * 3, s_hi=(2.0,) * 3,
                                                    p_lo=(-np.inf,) * 3, p_hi=(np.inf,) * 3, **base))
    np.testing.assert_array_equal(vel["x"], both["x"])
    assert not np.array_equal(vel["x"], plain["x"])


def test_admm_frozen_limit_matches_slsqp():
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc, nrm = _side_pass()
    res = oracle.solve(p, sc, oracle.OracleOptions(normal_mode=oracle.NORMAL_FROZEN, rho=10.0, max_iter=5000,
                                                   eps_abs=1e-11, eps_rel=1e-11), normals=nrm)
    J, b, G, h = _monolithic_pieces(p, sc, nrm)
    n = J.shape[1]
    fun = lambda U: float(np.sum((J @ U - b) ** 2))
    jac = lambda U: 2.0 * J.T @ (J @ U - b)
    sol = scipy.optimize.minimize(fun, np.zeros(n), jac=jac, method="SLSQP",
                                  bounds=[(-p.u_max, p.u_max)] * n,
                                  constraints=[dict(type="ineq", fun=lambda U: G @ U - h, jac=lambda U: G)],
                                  options=dict(ftol=1e-12, maxiter=2000))
    # SLSQP may end on its own line-search precision limit; its point must
    # still be feasible and agree with the ADMM limit, which must be no worse.
    assert sol.status in (0, 8)
    assert np.all(G @ sol.x - h >= -1e-8)
    np.testing.assert_allclose(res["u"].reshape(-1), sol.x, atol=1e-4)
    assert fun(res["u"].reshape(-1)) <= fun(sol.x) * (1 + 1e-9)


# ---------------------------------------------------------------------------
# The fallback normal of two coincident positions (Sec. III-A linearization;
# the reading: the reference relative position, else the relative reference
# velocity turned by 90 degrees (2-D) or crossed with the axis of its smallest
# component (3-D, ties to the lowest axis), else e_1).  Each case fixes the
# normal by geometric properties that determine it uniquely (unit length,
# perpendicularity, orientation), not by the oracle's formula.
# ---------------------------------------------------------------------------

def _coincident_refs(rng, N, T, dp, vel):
    """References of N agents whose positions all coincide at every step (so
    the reference relative position is zero) with per-agent velocities vel
    [N][dp]; the linearization point x is the references themselves."""
    xr = np.zeros((N, T + 1, 2 * dp))
    base = rng.normal(size=(T + 1, dp))
    xr[:, :, :dp] = base[None]
    xr[:, :, dp:] = vel[:, None, :]
    return xr


def _fallback_normals(dp, vel, T=3, seed=0):
    p = synth.ProblemParams(dp=dp, u_max=2.0)
    N = vel.shape[0]
    xr = _coincident_refs(np.random.default_rng(seed), N, T, dp, vel)
    sc = synth.Scenario(starts=xr[:, 0, :dp].copy(), goals=xr[:, -1, :dp].copy(), T=T)
    x0 = xr[:, 0, :].copy()
    return p, oracle.relinearize(p, sc, xr, inputs=(x0, xr))


def test_fallback_normal_2d_turns_the_relative_velocity_counterclockwise():
    """Coincident positions and coincident references, distinct reference
    velocities: n is the unit vector perpendicular to dv = v_i - v_j with
    det[dv, n] > 0 (dv turned counter-clockwise), the same at every step."""
    rng = np.random.default_rng(21)
    vel = rng.normal(size=(5, 2)) * 3.0
    p, n = _fallback_normals(2, vel)
    k = 0
    for i in range(5):
        for j in range(i + 1, 5):
            dv = vel[i] - vel[j]
            for t in range(n.shape[1]):
                m = n[k, t]
                assert np.linalg.norm(m) == pytest.approx(1.0, abs=1e-14)
                assert abs(m @ dv) <= 1e-13 * np.linalg.norm(dv)
                assert dv[0] * m[1] - dv[1] * m[0] > 0.5 * np.linalg.norm(dv)
            k += 1


def test_fallback_normal_3d_crosses_the_smallest_velocity_axis():
    """3-D: n is perpendicular to dv and to e_k, k the axis of the smallest
    |dv_k|, unit, with det[dv, e_k, n] > 0 (n along dv x e_k)."""
    rng = np.random.default_rng(22)
    vel = rng.normal(size=(6, 3)) * 2.0
    p, n = _fallback_normals(3, vel)
    k = 0
    for i in range(6):
        for j in range(i + 1, 6):
            dv = vel[i] - vel[j]
            kmin = int(np.argmin(np.abs(dv)))
            assert np.sort(np.abs(dv))[1] > np.abs(dv)[kmin] * (1 + 1e-9)   # no tie here
            e = np.eye(3)[kmin]
            for t in range(n.shape[1]):
                m = n[k, t]
                assert np.linalg.norm(m) == pytest.approx(1.0, abs=1e-14)
                assert abs(m @ dv) <= 1e-13 * np.linalg.norm(dv)
                assert m[kmin] == 0.0
                assert np.linalg.det(np.stack([dv, e, m])) > 0.0
            k += 1


def test_fallback_normal_3d_ties_go_to_the_lowest_axis():
    """dv = (0, 0, c): axes 0 and 1 tie at |dv_k| = 0, axis 0 wins, so n is
    perpendicular to e_0 and dv: n = sign(c) e_1 by the orientation rule;
    dv = (a, a, b) with |b| > |a|: axis 0, n = sign(...) in the plane
    perpendicular to e_0 and dv."""
    vel = np.array([[0.0, 0.0, 1.5], [0.0, 0.0, 0.0], [0.7, 0.7, -2.0], [0.0, 0.0, 0.0]])
    p, n = _fallback_normals(3, vel)
    # pair (0, 1): dv = (0, 0, 1.5)
    np.testing.assert_allclose(n[0, 0], [0.0, 1.0, 0.0], atol=1e-15)
    # pair (2, 3) (index 5 of 6): dv = (0.7, 0.7, -2); axis 0 (tie with 1)
    dv = vel[2] - vel[3]
    m = n[5, 0]
    assert m[0] == 0.0 and abs(m @ dv) <= 1e-14
    assert np.linalg.det(np.stack([dv, np.eye(3)[0], m])) > 0.0


@pytest.mark.parametrize("dp", [2, 3])
def test_fallback_normal_is_e1_without_relative_motion(dp):
    """Coincident positions, references and reference velocities: e_1."""
    vel = np.tile(np.array([[0.3, -1.2, 0.8][:dp]]), (3, 1))
    p, n = _fallback_normals(dp, vel)
    e1 = np.eye(dp)[0]
    for k in range(3):
        np.testing.assert_array_equal(n[k], np.tile(e1, (n.shape[1], 1)))


def test_fallback_normal_reference_position_first():
    """References apart at a step, positions coincident: the normalized
    reference relative position r_i - r_j (not the velocity rule)."""
    rng = np.random.default_rng(23)
    dp, N, T = 3, 4, 4
    vel = rng.normal(size=(N, dp))
    xr = _coincident_refs(rng, N, T, dp, vel)
    xr[:, 2, :dp] += rng.normal(size=(N, dp))          # step 2: references apart
    p = synth.ProblemParams(dp=dp, u_max=2.0)
    sc = synth.Scenario(starts=xr[:, 0, :dp].copy(), goals=xr[:, -1, :dp].copy(), T=T)
    x = xr.copy()
    x[:, :, :dp] = 0.0                                     # every position coincident
    n = oracle.relinearize(p, sc, x, inputs=(xr[:, 0, :].copy(), xr))
    k = 0
    for i in range(N):
        for j in range(i + 1, N):
            d = xr[i, 2, :dp] - xr[j, 2, :dp]
            assert n[k, 1] @ d == pytest.approx(np.linalg.norm(d), rel=1e-13)
            assert np.linalg.norm(n[k, 1]) == pytest.approx(1.0, abs=1e-14)
            k += 1


def test_frozen_reference_normals_of_an_exact_swap_use_the_velocity_rule():
    """The unjittered two-agent swap (both references pass the origin at
    t = T/2): a frozen solve with the oracle's own reference normals equals
    one given the normals of the linearization at the references, and the
    mid-horizon normal is perpendicular to the swap axis."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc = synth.circle_swap(2, 3.0, 20, 0.0, None)
    xr = sc.xref()
    assert np.all(xr[0, 10, :2] == xr[1, 10, :2])
    n = oracle.relinearize(p, sc, xr)
    dv = xr[0, 10, 2:] - xr[1, 10, 2:]
    assert abs(n[0, 9] @ dv) <= 1e-12 and dv[0] * n[0, 9, 1] - dv[1] * n[0, 9, 0] > 0
    o = oracle.OracleOptions(normal_mode=oracle.NORMAL_FROZEN, max_iter=80)
    a = oracle.solve(p, sc, o)
    b = oracle.solve(p, sc, o, normals=n)
    np.testing.assert_array_equal(a["x"], b["x"])
    np.testing.assert_array_equal(a["pair_active"], b["pair_active"])


def test_admm_point_symmetry():
    """Point-symmetric data and normal e_y: the solution is point symmetric,
    p_1(t) = -p_0(t), which checks the pair indexing and the signs of the
    consensus and dual updates."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc, nrm = _side_pass()
    res = oracle.solve(p, sc, oracle.OracleOptions(normal_mode=oracle.NORMAL_FROZEN, fixed_iters=60), normals=nrm)
    np.testing.assert_allclose(res["x"][1], -res["x"][0], atol=1e-12)
    np.testing.assert_allclose(res["u"][1], -res["u"][0], atol=1e-12)


def test_admm_duals_antisymmetric_and_along_normal():
    """Derived from Eqs. (4)-(5) under the projection reading:
    lambda_ij = -lambda_ji = -(rho/2) max(0, v) n after every update."""
    p, scs = synth.config2(S=1)
    sc = scs[0]
    res = oracle.solve(p, sc, oracle.OracleOptions(fixed_iters=30), keep_zl=True)
    lam, x = res["lam"], res["x"]
    N = sc.N
    np.testing.assert_allclose(lam + lam.transpose(1, 0, 2, 3), 0.0, atol=1e-12)
    for i in range(N):
        for j in range(i + 1, N):
            d = x[i, 1:, :2] - x[j, 1:, :2]
            n = d / np.linalg.norm(d, axis=1, keepdims=True)
            l = lam[i, j]
            cross = l[:, 0] * n[:, 1] - l[:, 1] * n[:, 0]
            np.testing.assert_allclose(cross, 0.0, atol=1e-9)
            assert np.all(np.sum(l * n, axis=1) <= 1e-12)


def test_admm_consensus_copies_satisfy_half_planes():
    """Every consensus pair (z_ij, z_ji) lies in its half-plane."""
    p, scs = synth.config2(S=2)
    sc = scs[1]
    res = oracle.solve(p, sc, oracle.OracleOptions(fixed_iters=25), keep_zl=True)
    z, x = res["z"], res["x"]
    for i in range(sc.N):
        for j in range(i + 1, sc.N):
            d = x[i, 1:, :2] - x[j, 1:, :2]
            n = d / np.linalg.norm(d, axis=1, keepdims=True)
            assert np.all(np.sum(n * (z[i, j] - z[j, i]), axis=1) >= p.d_min - 1e-12)


def test_admm_residual_history_consistent_with_iterates():
    """The residual recorded at iteration K+1 equals ||A x - z|| and
    rho ||A'(z^(K+1) - z^K)|| computed from two separate runs (lockstep)."""
    p, scs = synth.config2(S=1)
    sc = scs[0]
    K = 12
    a = oracle.solve(p, sc, oracle.OracleOptions(fixed_iters=K), keep_zl=True)
    b = oracle.solve(p, sc, oracle.OracleOptions(fixed_iters=K + 1), keep_zl=True)
    N, T = sc.N, sc.T
    r2 = s2 = 0.0
    for i in range(N):
        zs = np.zeros((T, 2))
        for j in range(N):
            if j == i:
                continue
            r2 += np.sum((b["x"][i, 1:, :2] - b["z"][i, j]) ** 2)
            zs += b["z"][i, j] - a["z"][i, j]
        s2 += np.sum((p.rho * zs) ** 2)
    np.testing.assert_allclose(b["hist"][K, 0], math.sqrt(r2), rtol=1e-10)
    np.testing.assert_allclose(b["hist"][K, 1], math.sqrt(s2), rtol=1e-10)
    np.testing.assert_allclose(b["hist"][:K], a["hist"][:K], rtol=0, atol=0)


def test_admm_single_agent_converges_first_iteration():
    p = synth.ProblemParams(dp=2)
    sc = synth.Scenario(starts=np.array([[0.0, 0.0]]), goals=np.array([[3.0, 1.0]]), T=20)
    res = oracle.solve(p, sc)
    assert res["status"] == oracle.CONVERGED and res["iters"] == 1
    direct = oracle.agent_qp(p, 20, 0, sc.x0()[0], sc.xref()[0], p.q_diag, p.r_diag)
    np.testing.assert_allclose(res["u"][0], direct["u"], atol=1e-12)


def test_admm_far_apart_agents_decouple():
    """No half-plane ever binds: the ADMM limit is each agent's own QP."""
    p = synth.ProblemParams(dp=2)
    sc = synth.Scenario(starts=np.array([[0.0, 0.0], [0.0, 20.0]]), goals=np.array([[3.0, 1.0], [-2.0, 21.0]]), T=20)
    res = oracle.solve(p, sc, oracle.OracleOptions(eps_abs=1e-11, eps_rel=1e-11, max_iter=3000))
    assert res["status"] == oracle.CONVERGED and not res["pair_active"].any()
    for i in range(2):
        direct = oracle.agent_qp(p, 20, 0, sc.x0()[i], sc.xref()[i], p.q_diag, p.r_diag)
        np.testing.assert_allclose(res["u"][i], direct["u"], atol=1e-8)


def _run_fixed(p, sc, K=40):
    return oracle.solve(p, sc, oracle.OracleOptions(fixed_iters=K))


def test_admm_translation_invariance():
    p, scs = synth.config2(S=1)
    sc = scs[0]
    c = np.array([1.7, -2.3])
    sh = copy.deepcopy(sc)
    sh.starts = sc.starts + c
    sh.goals = sc.goals + c
    a, b = _run_fixed(p, sc), _run_fixed(p, sh)
    np.testing.assert_allclose(b["x"][..., :2], a["x"][..., :2] + c, atol=1e-8)
    np.testing.assert_allclose(b["u"], a["u"], atol=1e-8)
    np.testing.assert_array_equal(b["w"], a["w"])


def test_admm_rotation_invariance():
    """A 90-degree rotation maps the input box onto itself."""
    p, scs = synth.config2(S=1)
    sc = scs[0]
    Rm = np.array([[0.0, -1.0], [1.0, 0.0]])
    ro = copy.deepcopy(sc)
    ro.starts = sc.starts @ Rm.T
    ro.goals = sc.goals @ Rm.T
    a, b = _run_fixed(p, sc), _run_fixed(p, ro)
    np.testing.assert_allclose(b["x"][..., :2], a["x"][..., :2] @ Rm.T, atol=1e-8)
    np.testing.assert_allclose(b["u"], a["u"] @ Rm.T, atol=1e-8)


def test_admm_permutation_invariance():
    p, scs = synth.config2(S=1)
    sc = scs[0]
    perm = np.random.default_rng(3).permutation(sc.N)
    pe = copy.deepcopy(sc)
    pe.starts = sc.starts[perm]
    pe.goals = sc.goals[perm]
    a, b = _run_fixed(p, sc), _run_fixed(p, pe)
    np.testing.assert_allclose(b["x"], a["x"][perm], atol=1e-8)
    np.testing.assert_array_equal(b["w"], a["w"][perm])


def test_admm_converged_solution_keeps_minimum_separation():
    """Fig. 3 property: a converged solve keeps every pair at least d_min
    apart (the half-planes are an inner approximation of the distance
    constraint), up to the primal tolerance."""
    p, scs = synth.config2(S=16)
    res = oracle.solve_batch(p, scs, threads=4)
    n_conv = 0
    for sc, r in zip(scs, res):
        if r["status"] != oracle.CONVERGED or sc.N < 2:
            continue
        n_conv += 1
        x = r["x"][:, 1:, :2]
        d = np.linalg.norm(x[:, None] - x[None], axis=-1)
        iu = np.triu_indices(sc.N, 1)
        assert d[iu].min() >= p.d_min - 2 * r["eps_pri"]
    assert n_conv >= 2


def test_admm_max_iter_and_cap_statuses():
    p, scs = synth.config1()
    r = oracle.solve(p, scs[0], oracle.OracleOptions(max_iter=1))
    assert r["status"] == oracle.MAX_ITER and r["iters"] == 1
    r = oracle.solve(p, scs[0], oracle.OracleOptions(max_as_iter=1))
    assert r["status"] == oracle.ACTIVE_SET_CAP and r["iters"] == 1


def test_admm_lu_reuse_changes_nothing():
    """The factor reuse keyed by the working set (the CPU mirror of the
    hotstart) is an optimisation only."""
    p, scs = synth.config2(S=1)
    a = oracle.solve(p, scs[0], oracle.OracleOptions(fixed_iters=20, lu_reuse=True))
    b = oracle.solve(p, scs[0], oracle.OracleOptions(fixed_iters=20, lu_reuse=False))
    np.testing.assert_allclose(a["x"], b["x"], atol=1e-9)
    assert a["lu_factorizations"] < b["lu_factorizations"]


# ---------------------------------------------------------------------------
# heterogeneous agents (per-agent weights and input boxes)
# ---------------------------------------------------------------------------

def _hetero_case(seed=3, N=4, T=12):
    p = synth.ProblemParams(dp=2, u_max=2.0)
    rng = np.random.default_rng(seed)
    sc = synth.random_box(rng, N, T)
    return p, synth.heterogeneous(rng, sc, p)


def test_hetero_single_agent_is_its_local_qp():
    """One agent alone converges in one iteration to its local QP: solved by
    the oracle's local QP routine with the agent's weights and box set
    problem-wide, the heterogeneous solve must agree."""
    p, sc = _hetero_case(N=3)
    one = dataclasses.replace(sc, starts=sc.starts[:1], goals=sc.goals[:1], agent_q=sc.agent_q[:1],
                              agent_r=sc.agent_r[:1], agent_lo=sc.agent_lo[:1], agent_hi=sc.agent_hi[:1])
    res = oracle.solve(p, one)
    assert res["status"] == oracle.CONVERGED and res["iters"] == 1
    umax = float(one.agent_hi[0, 0])
    p1 = dataclasses.replace(p, u_max=umax)
    # the local QP routine takes one symmetric box for all components: use
    # an agent whose two components share it
    one2 = dataclasses.replace(one, agent_lo=np.full((1, 2), -umax), agent_hi=np.full((1, 2), umax))
    res2 = oracle.solve(p, one2)
    o = oracle.agent_qp(p1, one.T, 0, one.x0()[0], one.xref()[0], one.agent_q[0], one.agent_r[0])
    np.testing.assert_allclose(res2["u"][0], o["u"], atol=1e-9)
    assert np.all(np.abs(res["u"][0]) <= one.agent_hi[0] + 1e-12)


def test_hetero_uniform_values_equal_the_scenario_solve():
    """Per-agent arrays that repeat the scenario's values change nothing."""
    p, scs = synth.config2(S=3)
    sc = scs[2]
    N = sc.N
    same = dataclasses.replace(sc, agent_q=np.tile(p.q_diag, (N, 1)), agent_r=np.tile(p.r_diag, (N, 1)),
                               agent_lo=np.tile(p.u_lo, (N, 1)), agent_hi=np.tile(p.u_hi, (N, 1)))
    o = oracle.OracleOptions(max_iter=40)
    a, b = oracle.solve(p, sc, o), oracle.solve(p, same, o)
    np.testing.assert_array_equal(a["x"], b["x"])
    np.testing.assert_array_equal(a["u"], b["u"])


def test_hetero_agent_permutation_equivariance():
    """Relabelling the agents together with their own weights and boxes
    relabels the solution (each agent's values follow it)."""
    p, sc = _hetero_case(seed=5, N=4, T=12)
    perm = np.array([2, 0, 3, 1])
    sp = dataclasses.replace(sc, starts=sc.starts[perm], goals=sc.goals[perm], agent_q=sc.agent_q[perm],
                             agent_r=sc.agent_r[perm], agent_lo=sc.agent_lo[perm], agent_hi=sc.agent_hi[perm])
    o = oracle.OracleOptions(max_iter=60)
    a, b = oracle.solve(p, sc, o), oracle.solve(p, sp, o)
    np.testing.assert_allclose(b["x"], a["x"][perm], atol=1e-9)
    # and the agents do differ: the weights matter
    hom = oracle.solve(p, dataclasses.replace(sc, agent_q=None, agent_r=None, agent_lo=None, agent_hi=None), o)
    assert np.abs(hom["u"] - a["u"]).max() > 1e-3


@pytest.mark.parametrize("alpha", [0.6, 1.0, 1.5, 1.9])
def test_admm_relaxation_closed_form_far_apart(alpha):
    """Over-relaxation (Boyd et al. 2011, Sec. 3.4.3) on two agents that
    never come near each other, with T = 1 and inactive input bounds.  Every
    projection is then the identity, so lambda stays 0 and z^(k+1) =
    alpha p^(k+1) + (1 - alpha) z^k, and each agent-axis local QP is a
    scalar quadratic in u_0 whose minimiser makes p_1 affine in z:
    p_1 = l z + beta with l = rho h^2 / H (h = B's position entry, H the
    second derivative).  After K iterations the oracle's p_1 and z must be
    those of this scalar recursion, started from z^0 = the reference."""
    p = synth.ProblemParams(dp=2, u_max=1e4)
    sc = synth.Scenario(starts=np.array([[-50.0, 3.0], [60.0, -40.0]]),
                        goals=np.array([[-48.0, 4.5], [58.0, -41.0]]), T=1)
    K, rho = 7, p.rho
    res = oracle.solve(p, sc, oracle.OracleOptions(alpha=alpha, fixed_iters=K), keep_zl=True)
    assert res["iters"] == K
    np.testing.assert_array_equal(res["lam"], 0.0)
    A, B = p.A, p.B
    dt, dp = p.dt, p.dp
    qT = p.qT_scale
    xr = sc.xref()
    for i in range(2):
        for c in range(dp):
            h, b = B[c, c], B[dp + c, c]           # position and velocity entries of B
            P = A[c] @ sc.x0()[i]                  # position after one step with u = 0
            V = A[dp + c] @ sc.x0()[i]
            rp, rv = xr[i, 1, c], xr[i, 1, dp + c]
            qp, qv, r = p.q_diag[c], p.q_diag[dp + c], p.r_diag[c]
            # d/du of qT qp (P + h u - rp)^2 + qT qv (V + b u - rv)^2 + r u^2 + rho/2 (P + h u - z)^2
            H = 2 * qT * qp * h * h + 2 * qT * qv * b * b + 2 * r + rho * h * h
            z = rp
            for _ in range(K):
                u = -(2 * qT * qp * h * (P - rp) + 2 * qT * qv * b * (V - rv) + rho * h * (P - z)) / H
                p1 = P + h * u
                z = alpha * p1 + (1 - alpha) * z
            assert res["x"][i, 1, c] == pytest.approx(p1, rel=1e-12, abs=1e-12)
            assert res["u"][i, 0, c] == pytest.approx(u, rel=1e-10, abs=1e-12)
            np.testing.assert_allclose(res["z"][i, 1 - i, 0, c], z, rtol=1e-12, atol=1e-12)


def test_admm_relaxation_frozen_limit_is_the_same_kkt_point():
    """Relaxation changes the path, not the fixed point: with alpha = 1.6 the
    frozen side pass converges to the same point as plain ADMM, which passes
    the centralized-QP certificate (test above), and does so in fewer
    iterations (the speed-up Boyd et al. report for alpha in [1.5, 1.8])."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc, nrm = _side_pass()
    tight = dict(normal_mode=oracle.NORMAL_FROZEN, rho=10.0, max_iter=1000, eps_abs=1e-10, eps_rel=1e-10)
    plain = oracle.solve(p, sc, oracle.OracleOptions(**tight), normals=nrm)
    relax = oracle.solve(p, sc, oracle.OracleOptions(alpha=1.6, **tight), normals=nrm)
    assert plain["status"] == oracle.CONVERGED and relax["status"] == oracle.CONVERGED
    np.testing.assert_allclose(relax["u"], plain["u"], atol=1e-7)
    np.testing.assert_allclose(relax["x"], plain["x"], atol=1e-7)
    assert relax["iters"] < plain["iters"]


class _WithDynamics:
    """A problem's constants with its dynamics replaced by (A, B)."""

    def __init__(self, p, A, B):
        for k in ("dp", "nx", "nu", "dt", "max_iter", "u_lo", "u_hi", "u_max", "q_diag", "r_diag", "qT_scale",
                  "d_min", "rho", "eps_abs", "eps_rel"):
            setattr(self, k, getattr(p, k))
        self.A, self.B = np.asarray(A, np.float64), np.asarray(B, np.float64)


def _mixed_case(seed=3, N=4, T=14):
    p, scs = synth.config2(S=40)
    sc = [s for s in scs if s.N >= N][0]
    sc = dataclasses.replace(sc, starts=sc.starts[:N], goals=sc.goals[:N], T=T)
    return p, synth.mixed_dynamics(np.random.default_rng(seed), sc, p)


def test_agent_dynamics_satisfied_per_agent():
    """Each agent's trajectory obeys its own dynamics x_{t+1} = A_i x_t +
    B_i u_t from its start, and its own are not its neighbours'."""
    p, sc = _mixed_case()
    res = oracle.solve(p, sc, oracle.OracleOptions(max_iter=60))
    for i in range(sc.N):
        x, u = res["x"][i], res["u"][i]
        np.testing.assert_allclose(x[0], sc.x0()[i], atol=0)
        pred = x[:-1] @ sc.agent_A[i].T + u @ sc.agent_B[i].T
        np.testing.assert_allclose(x[1:], pred, atol=1e-10)
        j = (i + 1) % sc.N
        other = x[:-1] @ sc.agent_A[j].T + u @ sc.agent_B[j].T
        assert np.abs(other - x[1:]).max() > 1e-6


def test_agent_dynamics_single_agent_is_its_local_qp():
    """One agent alone with its own dynamics converges in one iteration to
    the local QP solved with those dynamics set problem-wide."""
    p, sc = _mixed_case(N=3)
    one = dataclasses.replace(sc, starts=sc.starts[:1], goals=sc.goals[:1], agent_A=sc.agent_A[:1],
                              agent_B=sc.agent_B[:1])
    res = oracle.solve(p, one)
    assert res["status"] == oracle.CONVERGED and res["iters"] == 1
    o = oracle.agent_qp(_WithDynamics(p, one.agent_A[0], one.agent_B[0]), one.T, 0, one.x0()[0], one.xref()[0],
                        p.q_diag, p.r_diag)
    np.testing.assert_allclose(res["u"][0], o["u"], atol=1e-9)
    shared = oracle.solve(p, dataclasses.replace(one, agent_A=None, agent_B=None))
    assert np.abs(shared["u"][0] - o["u"]).max() > 1e-3


def test_agent_dynamics_uniform_equal_the_shared():
    """Per-agent dynamics that repeat the problem's change nothing."""
    p, scs = synth.config2(S=3)
    sc = scs[2]
    same = dataclasses.replace(sc, agent_A=np.tile(p.A, (sc.N, 1, 1)), agent_B=np.tile(p.B, (sc.N, 1, 1)))
    o = oracle.OracleOptions(max_iter=40)
    a, b = oracle.solve(p, sc, o), oracle.solve(p, same, o)
    np.testing.assert_array_equal(a["x"], b["x"])
    np.testing.assert_array_equal(a["u"], b["u"])


def test_agent_input_gain_is_a_reparametrization():
    """An agent whose input enters with gain g (B_i = g B) is the same agent
    with input v = g u: its R scaled by 1/g^2 and its box by g.  Through
    ADMM (4 crossing agents, 30 iterations in lockstep) the two give the
    same states, and the inputs differ by the gain."""
    p, sc = _mixed_case(N=4)
    g = np.array([0.5, 1.7, 1.0, 2.3])
    gained = dataclasses.replace(sc, agent_A=np.tile(p.A, (4, 1, 1)), agent_B=g[:, None, None] * p.B[None])
    scaled = dataclasses.replace(sc, agent_A=None, agent_B=None, agent_r=p.r_diag[None, :] / g[:, None] ** 2,
                                 agent_lo=p.u_lo[None, :] * g[:, None], agent_hi=p.u_hi[None, :] * g[:, None])
    o = oracle.OracleOptions(fixed_iters=30)
    a, b = oracle.solve(p, gained, o), oracle.solve(p, scaled, o)
    np.testing.assert_allclose(a["x"], b["x"], atol=1e-8)
    np.testing.assert_allclose(a["u"] * g[:, None, None], b["u"], atol=1e-8)


def test_agent_dynamics_permutation_equivariance():
    p, sc = _mixed_case(seed=5, N=4, T=12)
    perm = np.array([2, 0, 3, 1])
    sp = dataclasses.replace(sc, starts=sc.starts[perm], goals=sc.goals[perm], agent_A=sc.agent_A[perm],
                             agent_B=sc.agent_B[perm])
    o = oracle.OracleOptions(max_iter=60)
    a, b = oracle.solve(p, sc, o), oracle.solve(p, sp, o)
    np.testing.assert_allclose(b["x"], a["x"][perm], atol=1e-9)


def _momentum_far_apart_model(p, sc, K, eta=0.999):
    """The fast ADMM with restart (Goldstein et al. 2014, Alg. 8) on two
    agents that never come near each other (T = 1, inactive input bounds):
    every projection is the identity, so the duals stay 0, z_k = p_1(zh_k)
    with p_1 affine in zh per agent and axis (as in the relaxation pin), the
    combined residual is c_k = rho sum (z_k - zh_k)^2 over the ordered
    copies, and zh follows the extrapolation / restart rule."""
    rho, dt, dp, qT = p.rho, p.dt, p.dp, p.qT_scale
    A, B, xr = p.A, p.B, sc.xref()
    ell, beta0 = [], []
    for i in range(2):
        for c in range(dp):
            h, b = B[c, c], B[dp + c, c]
            P, V = A[c] @ sc.x0()[i], A[dp + c] @ sc.x0()[i]
            rp, rv = xr[i, 1, c], xr[i, 1, dp + c]
            qp, qv, r = p.q_diag[c], p.q_diag[dp + c], p.r_diag[c]
            H = 2 * qT * qp * h * h + 2 * qT * qv * b * b + 2 * r + rho * h * h
            # p_1 = P + h u, u = -(g0 + rho h (P - zh)) / H
            g0 = 2 * qT * qp * h * (P - rp) + 2 * qT * qv * b * (V - rv)
            ell.append(rho * h * h / H)
            beta0.append(P - h * (g0 + rho * h * P) / H)
    ell, beta0 = np.array(ell), np.array(beta0)
    z0 = np.array([xr[i, 1, c] for i in range(2) for c in range(dp)])
    zh, zprev, a, cprev, restarts = z0.copy(), z0.copy(), 1.0, np.inf, 0
    for k in range(1, K + 1):
        z = ell * zh + beta0                  # z_k = p_1 (the projection is the identity)
        ck = rho * np.sum((z - zh) ** 2)      # one ordered copy per agent and axis
        if k == K:
            break
        if ck < eta * cprev:
            an = 0.5 * (1 + np.sqrt(1 + 4 * a * a))
            zh = z + (a - 1) / an * (z - zprev)
            a, cprev = an, ck
        else:
            zh, a, cprev = zprev.copy(), 1.0, cprev / eta
            restarts += 1
        zprev = z
    return z.reshape(2, dp), restarts


def test_admm_momentum_closed_form_far_apart():
    """The oracle's momentum run against the scalar model above after K
    iterations; the model restarts at least once on the way, so both the
    extrapolation and the restart rule are pinned.  A large penalty makes
    plain ADMM slow here (p_1's slope in zh near 1), so the iterates are
    still far from the limit and differ from plain ADMM's."""
    p = synth.ProblemParams(dp=2, u_max=1e4, rho=1e4)
    sc = synth.Scenario(starts=np.array([[-50.0, 3.0], [60.0, -40.0]]),
                        goals=np.array([[-48.0, 4.5], [58.0, -41.0]]), T=1)
    K = 25
    want, restarts = _momentum_far_apart_model(p, sc, K)
    assert restarts >= 1
    res = oracle.solve(p, sc, oracle.OracleOptions(momentum=True, fixed_iters=K), keep_zl=True)
    plain = oracle.solve(p, sc, oracle.OracleOptions(fixed_iters=K))
    assert np.abs(plain["x"][:, 1, :2] - want).max() > 1e-3
    np.testing.assert_array_equal(res["lam"], 0.0)
    for i in range(2):
        np.testing.assert_allclose(res["x"][i, 1, :2], want[i], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(res["z"][i, 1 - i, 0], want[i], rtol=1e-12, atol=1e-12)


def test_admm_momentum_frozen_limit_is_the_same_kkt_point():
    """Momentum changes the path, not the fixed point: the frozen side pass
    converges to the plain-ADMM limit (certified above)."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc, nrm = _side_pass()
    tight = dict(normal_mode=oracle.NORMAL_FROZEN, rho=10.0, max_iter=2000, eps_abs=1e-10, eps_rel=1e-10)
    plain = oracle.solve(p, sc, oracle.OracleOptions(**tight), normals=nrm)
    fast = oracle.solve(p, sc, oracle.OracleOptions(momentum=True, **tight), normals=nrm)
    assert plain["status"] == oracle.CONVERGED and fast["status"] == oracle.CONVERGED
    np.testing.assert_allclose(fast["u"], plain["u"], atol=1e-7)
    np.testing.assert_allclose(fast["x"], plain["x"], atol=1e-7)
