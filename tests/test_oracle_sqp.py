"""Pins of the oracle's SQP outer loop (oracle/sqp.py, the re-linearization
of Sec. III-A's half-planes under the stopping rule of Sec. V-A)."""
import math

import numpy as np
import pytest
from scipy.linalg import block_diag
from scipy.spatial.distance import pdist

import oracle
import synth
from oracle import sqp


def _random_traj(rng, N, T, nx, nu):
    return rng.normal(size=(N, T + 1, nx)), rng.normal(size=(N, T, nu)), rng.normal(size=(N, T + 1, nx))


def test_objective_equals_stacked_quadratic_form():
    """Eq. 1 as one quadratic form over the stacked trajectory, with the
    weight matrix assembled block by block (Q for t < T, Q_T = qT Q at T, R
    on the inputs)."""
    rng = np.random.default_rng(11)
    p = synth.ProblemParams(dp=2)
    N, T = 3, 5
    x, u, r = _random_traj(rng, N, T, p.nx, p.nu)
    Q, R = np.diag(p.q_diag), np.diag(p.r_diag)
    Wx = block_diag(*([Q] * T + [p.qT_scale * Q]))
    Wu = block_diag(*([R] * T))
    want = 0.0
    for i in range(N):
        e = (x[i] - r[i]).reshape(-1)
        uu = u[i].reshape(-1)
        want += e @ Wx @ e + uu @ Wu @ uu
    assert sqp.objective(p, x, u, r, p.q_diag, p.r_diag) == pytest.approx(want, rel=1e-13)


def test_objective_special_cases():
    """Zero on the references with no input; a terminal offset d of one
    coordinate costs qT q_k d^2; an input a at t < T costs r_a a^2."""
    p = synth.ProblemParams(dp=2)
    N, T = 2, 4
    r = np.random.default_rng(3).normal(size=(N, T + 1, p.nx))
    u = np.zeros((N, T, p.nu))
    assert sqp.objective(p, r, u, r, p.q_diag, p.r_diag) == 0.0
    x = r.copy()
    x[1, T, 2] += 0.3
    assert sqp.objective(p, x, u, r, p.q_diag, p.r_diag) == pytest.approx(p.qT_scale * p.q_diag[2] * 0.09)
    u[0, 1, 1] = 1.5
    assert sqp.objective(p, x, u, r, p.q_diag, p.r_diag) == pytest.approx(
        p.qT_scale * p.q_diag[2] * 0.09 + p.r_diag[1] * 2.25)


def test_min_separation_matches_pairwise_distances():
    rng = np.random.default_rng(5)
    N, T, dp = 5, 6, 3
    x = rng.normal(size=(N, T + 1, 2 * dp))
    want = min(pdist(x[:, t, :dp]).min() for t in range(1, T + 1))
    assert sqp.min_separation(x, dp) == pytest.approx(want, rel=1e-14)
    x[2, 0, :dp] = x[3, 0, :dp]          # step 0 (the starts) is not constrained
    assert sqp.min_separation(x, dp) == pytest.approx(want, rel=1e-14)
    assert sqp.min_separation(x[:1], dp) == math.inf


def test_relinearized_normals_are_the_unit_separation_directions():
    """n of pair (i < j) at step t is the unit vector with n'(p_i - p_j) =
    |p_i - p_j|, in lexicographic pair order, t = 1..T."""
    p, scs = synth.config2(S=3)
    sc = scs[2]
    rng = np.random.default_rng(7)
    x = rng.normal(size=(sc.N, sc.T + 1, p.nx)) * 3.0
    n = oracle.relinearize(p, sc, x)
    P = sc.N * (sc.N - 1) // 2
    assert n.shape == (P, sc.T, p.dp)
    k = 0
    for i in range(sc.N):
        for j in range(i + 1, sc.N):
            for t in range(1, sc.T + 1):
                d = x[i, t, :p.dp] - x[j, t, :p.dp]
                assert np.linalg.norm(n[k, t - 1]) == pytest.approx(1.0, abs=1e-14)
                assert n[k, t - 1] @ d == pytest.approx(np.linalg.norm(d), rel=1e-13)
            k += 1


def test_relinearize_at_the_references_gives_the_oracles_reference_normals():
    """Round 0 (no normals: the reference normals inside the C oracle) equals a
    frozen-normal solve with the normals re-linearized about the references,
    which also covers the coincident-position fallback."""
    p, scs = synth.config0()
    sc = scs[0]
    o = oracle.OracleOptions(normal_mode=oracle.NORMAL_FROZEN, max_iter=60)
    a = oracle.solve(p, sc, o)
    b = oracle.solve(p, sc, o, normals=oracle.relinearize(p, sc, sc.xref()))
    np.testing.assert_array_equal(a["x"], b["x"])
    xr = sc.xref().copy()
    xr[1, 5, :p.dp] = xr[0, 5, :p.dp]      # coincident at t = 5: the reference normal there
    n = oracle.relinearize(p, sc, xr)
    d = sc.xref()[0, 5, :p.dp] - sc.xref()[1, 5, :p.dp]
    np.testing.assert_allclose(n[0, 4], d / np.linalg.norm(d), rtol=1e-14)


def _fixed_point_gap(p, sc, res):
    """Largest change of a binding half-plane's normal between the normals
    the last round used and those of its own solution."""
    used = res["normals"] if res["normals"] is not None else oracle.relinearize(p, sc, sc.xref())
    own = oracle.relinearize(p, sc, res["x"])
    act = res["pair_active"].astype(bool)
    return float(np.abs(own - used)[act].max()) if act.any() else 0.0


def test_sqp_reaches_a_collision_free_fixed_point():
    """Config 0 and small crossings with tight ADMM tolerances: the loop
    stops by its rule, the solution is collision-free, and the last round's
    binding half-planes are (to the loop's tolerance) tangent to the
    separation circles of its own solution."""
    p0, s0 = synth.config0()
    p2, s2 = synth.config2(S=40)
    small = [s for s in s2 if s.N <= 8][:3]
    o = oracle.OracleOptions(max_iter=5000, eps_abs=1e-6, eps_rel=1e-6)
    for p, scs in ((p0, s0), (p2, small)):
        for sc, r in zip(scs, sqp.sqp_solve(p, scs, o, max_rounds=10)):
            assert r["converged"] and r["rounds"] >= 2 and r["status"] == oracle.CONVERGED
            assert r["min_sep"][-1] >= p.d_min - 1e-3
            J = r["objective"]
            assert abs(J[-1] - J[-2]) <= 1e-4 * abs(J[-1])
            assert _fixed_point_gap(p, sc, r) <= 5e-3


def test_sqp_without_relinearization_fails_the_fixed_point():
    """Planted mistake: every round reuses the reference normals.  The loop
    stops after round 1 (the objective does not change), but the binding
    half-planes are far from those of the solution."""
    p, scs = synth.config0()
    sc = scs[0]
    o = oracle.OracleOptions(max_iter=5000, eps_abs=1e-6, eps_rel=1e-6)
    ref_normals = oracle.relinearize(p, sc, sc.xref())
    orig = oracle.relinearize
    try:
        oracle.relinearize = lambda problem, s, x, inputs=None: ref_normals
        r = sqp.sqp_solve(p, [sc], o, max_rounds=10, sep_tol=1.0)[0]
    finally:
        oracle.relinearize = orig
    assert r["rounds"] == 2 and r["objective"][0] == r["objective"][1]
    assert _fixed_point_gap(p, sc, dict(r, normals=ref_normals)) > 5e-2
