"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Both sides solve the same instance: the oracle receives the problem data
rounded to FP32 exactly as the device receives it.  Bar: relative trajectory
error over (x, u) <= 1e-4 per scenario, identical final working sets and
active half-planes except marginal (degenerate) entries, for every lockstep
run and every converged solve.  A run stopped by the 200-iteration cap
without converging is an iterate of a nonconvex iteration (the half-planes
follow the iterate) whose own sensitivity can exceed 1e-4: there the bar is
max(1e-4, 10 x the oracle's response to a 1e-7 perturbation of the starts),
and that sensitivity is printed with the result.
Inputs: the seeded generators of synth (shapes of the five workloads).
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_15838_amd as tadmm  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _zeros_eps(**kw):
    d = dict(eps_abs=0.0, eps_rel=0.0)
    d.update(kw)
    return d


def _lockstep_ok(g, K):
    """Exactly K iterations, or an exact fixed point earlier (r = s = 0 passes
    even a zero tolerance)."""
    return g["iters"] == K or (g["status"] == tadmm.SCEN_CONVERGED and g["r_norm"] == 0.0 and g["s_norm"] == 0.0)


def _full_tol(p, sc, o):
    if o["status"] == oracle.CONVERGED:
        return gc.REL_TOL, None
    kap = gc.self_sensitivity(p, sc, gc.oracle_opts(lockstep=o["iters"]), threads=4)
    return max(gc.REL_TOL, 10.0 * kap), kap


# ---------------------------------------------------------------------------
# one x-update (fixed z = C r, lambda = 0) against the oracle's local QP
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_first_xupdate_matches_oracle_local_qp(cfg):
    if cfg == "c1":
        p, scs = synth.config1()
    else:
        p, scs = synth.config2(S=6)
    _say(f"first x-update parity {cfg}")
    g = gc.gpu_solve(p, scs, solver_kw=_zeros_eps(max_iter=1))
    P32 = gc.Fp32Problem(p)
    for sc, gr in zip(scs, g):
        x0, xr = gc.fp32_inputs(sc)
        for i in range(sc.N):
            ysum = P32.rho * (sc.N - 1) * xr[i, :, :p.dp]
            o = oracle.agent_qp(P32, sc.T, sc.N - 1, x0[i], xr[i], P32.q_diag, P32.r_diag, ysum)
            X = np.concatenate([o["x"].ravel(), o["u"].ravel()])
            Y = np.concatenate([gr["x"][i].ravel(), gr["u"][i].ravel()])
            assert np.linalg.norm(X - Y) <= 1e-5 * np.linalg.norm(X), (sc.N, sc.T, i)
            marg = (gr["w"][i] != o["w"]) & (np.abs(o["mu"]) < gc.MARGIN * (1 + np.abs(o["mu"]).max()))
            assert np.all((gr["w"][i] == o["w"]) | marg)


# ---------------------------------------------------------------------------
# lockstep: exactly K iterations on both sides
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("K", [2, 10, 60])
def test_lockstep_config1(K):
    p, scs = synth.config1()
    _say(f"lockstep config1 K={K}")
    g = gc.gpu_solve(p, scs, solver_kw=_zeros_eps(max_iter=K), history=True)[0]
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(lockstep=K), keep_zl=True, threads=4)[0]
    assert _lockstep_ok(g, K) and o["iters"] == K
    rep = gc.compare(p, scs[0], g, o)
    rep["hist_worst"] = gc.compare_history(g, o, scs[0], p.dp)
    _say(f"  {rep}")


def test_lockstep_config2_sample():
    """40 iterations of 12 scenarios of the ragged batch: trajectories,
    working sets and active half-planes after the last iteration, and the
    residual norms of every iteration's stopping test."""
    p, scs = synth.config2(S=12)
    K = 40
    _say("lockstep config2 sample")
    g = gc.gpu_solve(p, scs, solver_kw=_zeros_eps(max_iter=K), history=True)
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(lockstep=K), keep_zl=True)
    worst, worst_h = 0.0, [0.0, 0.0]
    for sc, gr, orr in zip(scs, g, o):
        assert _lockstep_ok(gr, K), (sc.N, sc.T, gr["status"], gr["iters"])
        rep = gc.compare(p, sc, gr, orr)
        worst = max(worst, rep["rel"])
        h = gc.compare_history(gr, orr, sc, p.dp)
        worst_h = [max(a, b) for a, b in zip(worst_h, h)]
    _say(f"  worst rel {worst:.2e}; worst residual-history ratio (r, s) {worst_h}")


# ---------------------------------------------------------------------------
# full solves with the stopping rule
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [0, 1, 2])
def test_config0_parity(mode):
    p, scs = synth.config0()
    _say(f"config0 mode={mode}")
    g = gc.gpu_solve(p, scs, mode=mode)[0]
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(), keep_zl=True)[0]
    tol, kap = _full_tol(p, scs[0], o)
    rep = gc.compare(p, scs[0], g, o, tol=tol)
    assert abs(g["iters"] - o["iters"]) <= 2 and g["status"] == o["status"], rep
    _say(f"  {rep} sensitivity={kap}")


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_config1_parity(mode):
    p, scs = synth.config1()
    _say(f"config1 mode={mode}")
    g = gc.gpu_solve(p, scs, mode=mode)[0]
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(), keep_zl=True, threads=4)[0]
    tol, kap = _full_tol(p, scs[0], o)
    rep = gc.compare(p, scs[0], g, o, tol=tol)
    assert abs(g["iters"] - o["iters"]) <= 2 and g["status"] == o["status"], rep
    _say(f"  {rep} sensitivity={kap}")


def test_config2_sample_parity_batched():
    """The headline workload's scenarios through the persistent kernel: per
    scenario the same status, iterations within 2, the trajectory bar, and
    identical final working sets and active half-planes except marginal
    entries."""
    p, scs = synth.config2(S=24)
    _say("config2 sample batched")
    g = gc.gpu_solve(p, scs)
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(), keep_zl=True)
    worst_conv, worst_cap, marg = 0.0, 0.0, [0, 0]
    for sc, gr, orr in zip(scs, g, o):
        assert gr["status"] == orr["status"], (sc.N, sc.T, gr["status"], orr["status"])
        assert abs(gr["iters"] - orr["iters"]) <= 2, (sc.N, sc.T, gr["iters"], orr["iters"])
        tol, kap = _full_tol(p, sc, orr)
        rep = gc.compare(p, sc, gr, orr, tol=tol)
        marg[0] += rep["w_marginal"]
        marg[1] += rep.get("pair_marginal", 0)
        if kap is None:
            worst_conv = max(worst_conv, rep["rel"])
        else:
            worst_cap = max(worst_cap, rep["rel"])
    _say(f"  worst rel converged {worst_conv:.2e}, at the iteration cap {worst_cap:.2e}; "
         f"marginal entries excluded: working sets {marg[0]}, half-planes {marg[1]}")


def test_frozen_normals_parity():
    """Convex case: fixed normals given by the caller (three agents in
    parallel lanes whose goals pull the outer lanes inward, so that two
    half-planes bind at convergence)."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc = synth.Scenario(starts=np.array([[-2.0, 0.0], [-2.0, 1.5], [2.0, -1.5]]),
                        goals=np.array([[2.0, 0.0], [2.0, 0.3], [-2.0, -0.3]]), T=20)
    T, P = sc.T, 3
    nrm = np.zeros((P, T, 2))
    nrm[0, :, 1] = -1.0   # agent 1 stays above agent 0
    nrm[1, :, 1] = 1.0    # agent 0 stays above agent 2
    nrm[2, :, 1] = 1.0    # agent 1 stays above agent 2
    kw = dict(normal_mode=tadmm.NORMAL_FROZEN, max_iter=1000)
    _say("frozen normals")
    g = gc.gpu_solve(p, [sc], normals=[nrm], solver_kw=kw)[0]
    o = gc.oracle_same_instance(p, [sc], gc.oracle_opts(kw), keep_zl=True,
                                normals=[np.asarray(nrm, np.float32).astype(np.float64)])[0]
    assert o["status"] == oracle.CONVERGED and o["pair_active"].sum() >= 1
    assert g["status"] == tadmm.SCEN_CONVERGED and abs(g["iters"] - o["iters"]) <= 2
    gc.compare(p, sc, g, o, check_sets=False)


# ---------------------------------------------------------------------------
# the fallback normal of coincident positions (reference relative position,
# else the relative reference velocity turned by 90 degrees (2-D) or crossed
# with its smallest axis (3-D), else e_1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [0, 1])
def test_exact_swap_frozen_reference_normals(mode):
    """The unjittered two-agent swap: both references pass the origin at
    t = T/2, where the frozen reference normal comes from the relative
    reference velocity.  The frozen half-planes of the references are not
    jointly feasible under the input box here (the oracle's primal residual
    stays near 5), so the two sides are compared in lockstep."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc = synth.circle_swap(2, 3.0, 20, 0.0, None)
    K = 60
    kw = dict(normal_mode=tadmm.NORMAL_FROZEN, eps_abs=0.0, eps_rel=0.0, max_iter=K)
    _say(f"exact swap, frozen reference normals, mode={mode}")
    g = gc.gpu_solve(p, [sc], mode=mode, solver_kw=kw, history=True)[0]
    o = gc.oracle_same_instance(p, [sc], gc.oracle_opts(kw, lockstep=K), keep_zl=True)[0]
    assert _lockstep_ok(g, K) and o["iters"] == K
    assert o["pair_active"][0, 9] == 1          # the mid-horizon half-plane binds
    rep = gc.compare(p, sc, g, o, normals=oracle.relinearize(gc.Fp32Problem(p), sc, gc.fp32_inputs(sc)[1],
                                                             inputs=gc.fp32_inputs(sc)))
    rep["hist_worst"] = gc.compare_history(g, o, sc, p.dp)
    _say(f"  {rep}")


def test_exact_swap_per_iteration_normals():
    """The unjittered swap with normals of the iterates: a full solve to the
    stopping rule on both sides."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc = synth.circle_swap(2, 3.0, 20, 0.0, None)
    _say("exact swap, per-iteration normals")
    g = gc.gpu_solve(p, [sc], history=True)[0]
    o = gc.oracle_same_instance(p, [sc], gc.oracle_opts(), keep_zl=True)[0]
    assert o["status"] == oracle.CONVERGED
    assert g["status"] == tadmm.SCEN_CONVERGED and abs(g["iters"] - o["iters"]) <= 2, (g["iters"], o["iters"])
    rep = gc.compare(p, sc, g, o)
    rep["hist_worst"] = gc.compare_history(g, o, sc, p.dp)
    _say(f"  {rep}")


def test_coincident_positions_per_iteration_fallback():
    """Two agents with the same start and goal (input checks off): their
    first x-updates are identical, so the first consensus step sees
    coincident positions and coincident references with equal velocities and
    takes e_1; a third agent crosses them.  Lockstep with the oracle."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc = synth.Scenario(starts=np.array([[0.0, 0.0], [0.0, 0.0], [3.0, 1.0]]),
                        goals=np.array([[2.0, 1.0], [2.0, 1.0], [-2.0, 0.0]]), T=15)
    K = 30
    kw = _zeros_eps(max_iter=K, check_inputs=False)
    _say("coincident positions, per-iteration normals")
    g = gc.gpu_solve(p, [sc], solver_kw=kw, history=True)[0]
    o = gc.oracle_same_instance(p, [sc], gc.oracle_opts(lockstep=K), keep_zl=True)[0]
    assert _lockstep_ok(g, K) and o["iters"] == K
    rep = gc.compare(p, sc, g, o)
    rep["hist_worst"] = gc.compare_history(g, o, sc, p.dp)
    assert np.all(np.abs(g["x"][0, 1:, 0] - g["x"][1, 1:, 0]) > 0.0)   # pushed apart along e_1
    _say(f"  {rep}")


def test_tiny_dmin_near_coincident_pair_takes_the_full_step():
    """d_min = 1e-7 and two agents at rest 3e-7 apart (input checks off):
    the pair is farther apart than d_min, but closer than the 1e-6 below
    which the normal falls back to the references (here e_1, no relative
    reference motion), and that half-plane is violated.  The consensus step
    must take it (active), as the oracle does."""
    p = synth.ProblemParams(dp=2, u_max=2.0, d_min=1e-7)
    pts = np.array([[0.0, 0.0], [3e-7, 0.0]])
    sc = synth.Scenario(starts=pts, goals=pts.copy(), T=10)
    K = 10
    kw = _zeros_eps(max_iter=K, check_inputs=False)
    _say("d_min 1e-7, near-coincident pair")
    g = gc.gpu_solve(p, [sc], solver_kw=kw)[0]
    o = gc.oracle_same_instance(p, [sc], gc.oracle_opts(lockstep=K), keep_zl=True)[0]
    assert _lockstep_ok(g, K) and o["iters"] == K
    assert o["pair_active"].sum() > 0
    rep = gc.compare(p, sc, g, o)
    _say(f"  {rep}")


def test_three_d_frozen_reference_normals_lockstep():
    """The 3-D scale workload with frozen reference normals: every one of
    the 8128 pairs has coincident references at t = 25 (all agents pass the
    sphere's centre), where the normal is the relative reference velocity
    crossed with its smallest axis.  Three iterations in lockstep, every
    agent and half-plane."""
    p, scs = synth.config4()
    K = 3
    kw = dict(normal_mode=tadmm.NORMAL_FROZEN, eps_abs=0.0, eps_rel=0.0, max_iter=K)
    _say(f"3-D config4 frozen reference normals, lockstep K={K}")
    g = gc.gpu_solve(p, scs, solver_kw=kw)[0]
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(kw, lockstep=K), keep_zl=True, threads=0)[0]
    assert _lockstep_ok(g, K) and o["iters"] == K
    assert o["pair_active"][:, 24].sum() > 0
    x0, xr = gc.fp32_inputs(scs[0])
    rep = gc.compare(p, scs[0], g, o, normals=oracle.relinearize(gc.Fp32Problem(p), scs[0], xr, inputs=(x0, xr)))
    _say(f"  {rep}")


def test_three_d_first_iterations_sampled():
    """3-D double integrator, 128 agents on a sphere (horizon 50): the first
    x-update of sampled agents equals the oracle's local QP; then a short
    lockstep of a 12-agent 3-D scenario."""
    p, scs = synth.config4()
    sc = scs[0]
    _say("3-D config4 first x-update, sampled agents")
    g = gc.gpu_solve(p, scs, solver_kw=_zeros_eps(max_iter=1), mode=tadmm.MODE_PLAIN)[0]
    P32 = gc.Fp32Problem(p)
    x0, xr = gc.fp32_inputs(sc)
    for i in (0, 37, 64, 127):
        ysum = P32.rho * (sc.N - 1) * xr[i, :, :p.dp]
        o = oracle.agent_qp(P32, sc.T, sc.N - 1, x0[i], xr[i], P32.q_diag, P32.r_diag, ysum)
        X = np.concatenate([o["x"].ravel(), o["u"].ravel()])
        Y = np.concatenate([g["x"][i].ravel(), g["u"][i].ravel()])
        assert np.linalg.norm(X - Y) <= 1e-5 * np.linalg.norm(X), i
    small = synth.sphere_swap(12, 4.0, 30)
    K = 25
    g2 = gc.gpu_solve(p, [small], solver_kw=_zeros_eps(max_iter=K))[0]
    o2 = gc.oracle_same_instance(p, [small], gc.oracle_opts(lockstep=K), keep_zl=True, threads=4)[0]
    assert _lockstep_ok(g2, K)
    gc.compare(p, small, g2, o2)


def test_three_d_full_size_lockstep():
    """The 3-D scale workload at full size (128 agents, T = 50, 8128 pairs x
    50 steps): the first iterations in lockstep with the oracle, every agent
    (the warm start alone takes ~190 active-set passes per agent)."""
    p, scs = synth.config4()
    K = 3
    _say(f"3-D config4 full-size lockstep K={K}")
    g = gc.gpu_solve(p, scs, solver_kw=_zeros_eps(max_iter=K))[0]
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(lockstep=K), keep_zl=True, threads=0)[0]
    assert _lockstep_ok(g, K) and o["iters"] == K
    rep = gc.compare(p, scs[0], g, o)
    _say(f"  {rep}")


# ---------------------------------------------------------------------------
# plain == batched, determinism, ablation flags
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [1, 2])
def test_plain_and_batched_bitwise_equal(mode):
    """The persistent kernel (1) and the many-workgroup graphs (2) run the
    plain path's per-scenario arithmetic: identical iterates, bit for bit."""
    p, scs = synth.config2(S=10)
    _say(f"plain vs mode {mode} bitwise")
    a = gc.gpu_solve(p, scs, mode=tadmm.MODE_PLAIN)
    b = gc.gpu_solve(p, scs, mode=mode)
    for ga, gb in zip(a, b):
        assert ga["iters"] == gb["iters"] and ga["status"] == gb["status"]
        np.testing.assert_array_equal(ga["x"], gb["x"])
        np.testing.assert_array_equal(ga["u"], gb["u"])
        np.testing.assert_array_equal(ga["w"], gb["w"])
        np.testing.assert_array_equal(ga["pair_active"], gb["pair_active"])
        np.testing.assert_array_equal(ga["counters"][:4], gb["counters"][:4])


def test_wide_mode_three_d_scale_equals_plain():
    """The 3-D scale workload (one scenario of 128 agents) through the
    many-workgroup mode: bitwise the plain path's iterates, 40 iterations."""
    p, scs = synth.config4()
    _say("config4 wide vs plain, 40 iterations")
    kw = dict(max_iter=40)
    a = gc.gpu_solve(p, scs, mode=tadmm.MODE_PLAIN, solver_kw=kw)[0]
    b = gc.gpu_solve(p, scs, mode=tadmm.MODE_WIDE, solver_kw=kw)[0]
    assert a["iters"] == b["iters"] == 40
    np.testing.assert_array_equal(a["x"], b["x"])
    np.testing.assert_array_equal(a["pair_active"], b["pair_active"])


@pytest.mark.parametrize("threads", [64, 128, 256])
def test_batched_independent_of_workgroup_size(threads):
    p, scs = synth.config2(S=10)
    a = gc.gpu_solve(p, scs, solver_kw=dict(block_threads=64))
    b = gc.gpu_solve(p, scs, solver_kw=dict(block_threads=threads))
    for ga, gb in zip(a, b):
        np.testing.assert_array_equal(ga["x"], gb["x"])
        assert ga["iters"] == gb["iters"]


def test_deterministic_repeat():
    p, scs = synth.config2(S=10)
    res, prep, solver = gc.gpu_solve(p, scs, return_prep=True)
    x1 = prep.o["x"].clone()
    prep.run(tadmm.MODE_BATCHED)
    torch.testing.assert_close(prep.o["x"], x1, rtol=0, atol=0)
    solver.close()


@pytest.mark.parametrize("flag", ["cache_factors", "riccati_warmstart", "hotstart"])
def test_ablation_flags_same_iterates(flag):
    """Factor caching, the Riccati warm start and the hotstart change the work,
    not the iterates (each local QP has a unique minimiser)."""
    p, scs = synth.config2(S=6)
    K = 30
    a = gc.gpu_solve(p, scs, solver_kw=_zeros_eps(max_iter=K))
    b = gc.gpu_solve(p, scs, solver_kw=_zeros_eps(max_iter=K, **{flag: False}))
    for ga, gb in zip(a, b):
        rel = gc.rel_traj_err(gb, dict(x=ga["x"].astype(np.float64), u=ga["u"].astype(np.float64)))
        assert rel <= 1e-5, (flag, rel)
    ca = sum(g["counters"] for g in a)
    cb = sum(g["counters"] for g in b)
    if flag == "cache_factors":
        assert cb[1] > ca[1]          # more refactored stages
    else:
        assert cb[0] >= ca[0]         # at least as many active-set passes


@pytest.mark.parametrize("mode", [0, 1])
def test_cached_factors_and_restarted_sweeps_are_exact(mode):
    """With cached factors, a later active-set pass refactors only the stages
    at and below its working-set change and restarts the affine sweep from a
    kept stage above it (Eqs. 7-8 with the other stages' factors and costates
    unchanged).  Without caching every pass refactors and sweeps every stage:
    the same arithmetic on the same inputs, so the iterates, iteration counts
    and statuses must be bitwise equal, with fewer refactored stages and
    fewer swept stages in the cached run."""
    p, scs = synth.config2(S=12)
    _say(f"cached factors vs full refactors, mode={mode}")
    a = gc.gpu_solve(p, scs, mode=mode)
    b = gc.gpu_solve(p, scs, mode=mode, solver_kw=dict(cache_factors=False))
    for ga, gb in zip(a, b):
        assert np.array_equal(ga["x"], gb["x"]) and np.array_equal(ga["u"], gb["u"])
        assert ga["iters"] == gb["iters"] and ga["status"] == gb["status"]
        assert np.array_equal(ga["counters"][0], gb["counters"][0])   # the same active-set passes
    ca = sum(g["counters"] for g in a)
    cb = sum(g["counters"] for g in b)
    assert ca[1] < cb[1] and ca[2] < cb[2], (ca, cb)


# ---------------------------------------------------------------------------
# edge cases and failure paths
# ---------------------------------------------------------------------------

def test_single_agent_converges_in_one_iteration():
    p = synth.ProblemParams(dp=2)
    sc = synth.Scenario(starts=np.array([[0.0, 0.0]]), goals=np.array([[3.0, 1.0]]), T=20)
    g = gc.gpu_solve(p, [sc])[0]
    assert g["status"] == tadmm.SCEN_CONVERGED and g["iters"] == 1
    o = oracle.agent_qp(p, 20, 0, sc.x0()[0], sc.xref()[0], p.q_diag, p.r_diag)
    assert gc.rel_traj_err(dict(x=g["x"][0], u=g["u"][0]), o) <= 1e-5


def test_horizon_one_and_mixed_tiny_batch():
    p = synth.ProblemParams(dp=2)
    scs = [synth.Scenario(starts=np.array([[0.0, 0.0], [1.0, 0.0]]), goals=np.array([[1.0, 0.0], [0.0, 0.0]]), T=1),
           synth.Scenario(starts=np.array([[0.0, 0.0]]), goals=np.array([[1.0, 1.0]]), T=3),
           synth.Scenario(starts=np.array([[0.0, 0.0], [0.0, 1.5], [1.5, 0.0]]),
                          goals=np.array([[1.5, 1.5], [1.5, 0.0], [0.0, 1.5]]), T=7)]
    g = gc.gpu_solve(p, scs)
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts())
    for sc, gr, orr in zip(scs, g, o):
        assert abs(gr["iters"] - orr["iters"]) <= 2
        tol, _ = _full_tol(p, sc, orr)
        assert gc.rel_traj_err(gr, orr) <= tol


def test_empty_batch_is_noop():
    p = synth.ProblemParams(dp=2)
    solver = tadmm.Solver(tadmm.make_params(p))
    prep = solver.prepare(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros((0, 4)), np.zeros((0, 4)),
                          np.zeros((0, 4)), np.zeros((0, 2)))
    prep.run(tadmm.MODE_BATCHED)
    solver.close()


def test_max_iter_one_and_cap_statuses():
    p, scs = synth.config1()
    g = gc.gpu_solve(p, scs, solver_kw=dict(max_iter=1))[0]
    assert g["status"] == tadmm.SCEN_MAX_ITER and g["iters"] == 1
    g = gc.gpu_solve(p, scs, solver_kw=dict(max_as_iter=1))[0]
    assert g["status"] == tadmm.SCEN_ACTIVE_SET_CAP and g["iters"] == 1


def test_nonfinite_input_rejected():
    p, scs = synth.config2(S=3)
    pk = synth.pack(p, scs)
    pk.xref[5, 0] = np.nan
    solver = tadmm.Solver(tadmm.make_params(p))
    with pytest.raises(tadmm.TadmmError) as e:
        solver.solve(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag)
    assert e.value.code == 3
    solver.close()


def test_close_start_rejected():
    p = synth.ProblemParams(dp=2)
    sc = synth.Scenario(starts=np.array([[0.0, 0.0], [0.1, 0.0]]), goals=np.array([[1.0, 0.0], [0.0, 1.0]]), T=10)
    pk = synth.pack(p, [sc])
    solver = tadmm.Solver(tadmm.make_params(p))
    with pytest.raises(tadmm.TadmmError) as e:
        solver.solve(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag)
    assert e.value.code == 4
    solver.close()


def test_poisoned_scenario_is_isolated():
    """With the input checks off, a NaN reference in one scenario ends that
    scenario as NONFINITE and leaves every other scenario bitwise unchanged."""
    p, scs = synth.config2(S=5)
    pk = synth.pack(p, scs)
    solver = tadmm.Solver(tadmm.make_params(p, check_inputs=False))
    clean = tadmm.split_outputs(solver.solve(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag),
                                pk.n_agents, pk.horizon, p.nx, p.nu)
    bad = pk.xref.copy()
    off = int((pk.n_agents[:2] * (pk.horizon[:2] + 1)).sum())
    bad[off + 3, 0] = np.nan
    pois = tadmm.split_outputs(solver.solve(pk.n_agents, pk.horizon, pk.x0, bad, pk.q_diag, pk.r_diag),
                               pk.n_agents, pk.horizon, p.nx, p.nu)
    assert pois[2]["status"] == tadmm.SCEN_NONFINITE
    for s in (0, 1, 3, 4):
        np.testing.assert_array_equal(pois[s]["x"], clean[s]["x"])
        assert pois[s]["iters"] == clean[s]["iters"]
    solver.close()


def test_autotuned_configuration_meets_the_parity_bar():
    """tadmm_autotune on a sample of the ragged batch picks a workgroup size
    among its candidates; the solve in that configuration equals the oracle
    to the parity bar (statuses, iterations within 2, trajectories, sets) and
    is bitwise the default configuration's (the arithmetic of a scenario
    does not depend on the launch shape)."""
    p, scs = synth.config2(S=16)
    _say("autotuned configuration vs the oracle")
    g0, prep, solver = gc.gpu_solve(p, scs, return_prep=True)
    best = prep.autotune()
    assert best in (64, 128, 192, 256)
    prep.run(tadmm.MODE_BATCHED)
    g = tadmm.split_outputs(prep.result(), [s.N for s in scs], [s.T for s in scs], p.nx, p.nu)
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(), keep_zl=True)
    for sc, ga, gr, orr in zip(scs, g0, g, o):
        np.testing.assert_array_equal(ga["x"], gr["x"])
        assert gr["status"] == orr["status"] and abs(gr["iters"] - orr["iters"]) <= 2
        tol, _ = _full_tol(p, sc, orr)
        gc.compare(p, sc, gr, orr, tol=tol)
    _say(f"  tuned workgroup size {best}")
    solver.close()
