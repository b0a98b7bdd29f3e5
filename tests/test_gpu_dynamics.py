"""Per-agent dynamics on the device (each agent a damped point mass of its
own drag and mass, exactly discretized) against the oracle, through the C
ABI.  The per-agent matrices are rounded to FP32 on the host, so both sides
solve the instance the device receives.  With them the device takes the
one-lane-per-agent path for every agent."""
import dataclasses
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


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _mixed(p, scs, seed):
    rng = np.random.default_rng(seed)
    out = []
    for sc in scs:
        m = synth.mixed_dynamics(rng, sc, p)
        out.append(dataclasses.replace(m, agent_A=_f32(m.agent_A), agent_B=_f32(m.agent_B)))
    return out


@pytest.mark.parametrize("dp", [2, 3])
def test_agent_dynamics_lockstep_matches_oracle(dp):
    if dp == 2:
        p, scs = synth.config2(S=12)
    else:
        p = synth.ProblemParams(dp=3, u_max=3.0)
        _, base = synth.config2(S=40)
        base = [s for s in base if s.N <= 12][:6]
        rng = np.random.default_rng(2)
        scs = [synth.Scenario(starts=np.concatenate([s.starts, rng.uniform(-5, 5, (s.N, 1))], 1),
                              goals=np.concatenate([s.goals, rng.uniform(-5, 5, (s.N, 1))], 1), T=s.T) for s in base]
    scs = _mixed(p, scs, seed=7 + dp)
    K = 40
    _say(f"per-agent dynamics lockstep, {dp}-D, K={K}, N = {[s.N for s in scs]}")
    g = gc.gpu_solve(p, scs, solver_kw=dict(max_iter=K, eps_abs=0.0, eps_rel=0.0))
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(lockstep=K), threads=4)
    worst = 0.0
    for sc, gr, orr in zip(scs, g, o):
        assert gr["iters"] == K or (gr["status"] == tadmm.SCEN_CONVERGED and gr["r_norm"] == 0.0
                                    and gr["s_norm"] == 0.0)
        rel = gc.rel_traj_err(gr, orr)
        worst = max(worst, rel)
        assert rel <= gc.REL_TOL, (sc.N, sc.T, rel)
        # each agent follows its own dynamics
        for i in range(sc.N):
            x, u = gr["x"][i].astype(np.float64), gr["u"][i].astype(np.float64)
            pred = x[:-1] @ sc.agent_A[i].T + u @ sc.agent_B[i].T
            assert np.abs(pred - x[1:]).max() <= 1e-4 * (1 + np.abs(x).max())
    _say(f"  worst rel {worst:.2e}")


def test_agent_dynamics_converged_solves_match_oracle():
    p, scs = synth.config2(S=24)
    scs = _mixed(p, scs, seed=11)
    g = gc.gpu_solve(p, scs)
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts())
    n = 0
    for sc, gr, orr in zip(scs, g, o):
        if orr["status"] != oracle.CONVERGED:
            continue
        n += 1
        assert gr["status"] == tadmm.SCEN_CONVERGED, (sc.N, sc.T)
        assert gc.rel_traj_err(gr, orr) <= gc.REL_TOL
    _say(f"  {n} converged scenarios compared")
    assert n >= 3


def test_uniform_agent_dynamics_take_the_general_path():
    """The shared double integrator given per agent runs one lane per agent
    instead of the per-axis split: the same QPs, so the results agree within
    the parity bar (not bitwise: the lane decompositions differ)."""
    p, scs = synth.config2(S=8)
    same = [dataclasses.replace(sc, agent_A=np.tile(p.A, (sc.N, 1, 1)), agent_B=np.tile(p.B, (sc.N, 1, 1)))
            for sc in scs]
    kw = dict(max_iter=40, eps_abs=0.0, eps_rel=0.0)
    a = gc.gpu_solve(p, scs, solver_kw=kw)
    b = gc.gpu_solve(p, same, solver_kw=kw)
    for ga, gb in zip(a, b):
        assert gc.rel_traj_err(ga, dict(x=gb["x"].astype(np.float64), u=gb["u"].astype(np.float64))) <= gc.REL_TOL


def test_agent_dynamics_modes_bitwise_equal():
    p, scs = synth.config2(S=10)
    scs = _mixed(p, scs, seed=3)
    kw = dict(max_iter=100)
    a = gc.gpu_solve(p, scs, mode=tadmm.MODE_PLAIN, solver_kw=kw)
    for mode in (tadmm.MODE_BATCHED, tadmm.MODE_WIDE):
        b = gc.gpu_solve(p, scs, mode=mode, solver_kw=kw)
        for ga, gb in zip(a, b):
            assert ga["iters"] == gb["iters"]
            np.testing.assert_array_equal(ga["x"], gb["x"])


def test_agent_dynamics_bad_inputs_and_derivative_rejected():
    p, scs = synth.config2(S=2)
    scs = _mixed(p, scs, seed=5)
    pk = synth.pack(p, scs)
    solver = tadmm.Solver(tadmm.make_params(p))
    bad = pk.agent_A.copy()
    bad[1, 3] = np.nan
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag, agent_A=bad,
                          agent_B=pk.agent_B)
    with pytest.raises(tadmm.TadmmError) as e:
        prep.run(tadmm.MODE_BATCHED)
    assert "error 3" in str(e.value)
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag, agent_A=pk.agent_A)
    with pytest.raises(tadmm.TadmmError) as e:
        prep.run(tadmm.MODE_BATCHED)
    assert "error 1" in str(e.value)
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag, agent_A=pk.agent_A,
                          agent_B=pk.agent_B)
    prep.run(tadmm.MODE_BATCHED)
    with pytest.raises(tadmm.TadmmError) as e:
        prep.polish()
    assert "error 1" in str(e.value)
    solver.close()


def test_agent_dynamics_with_box_relaxation_and_hetero_weights_lockstep():
    """Per-agent dynamics together with per-agent weights and boxes, the
    velocity box and over-relaxation, in lockstep with the oracle (the
    general path with every option that composes with it)."""
    p, scs = synth.config2(S=6)
    rng = np.random.default_rng(21)
    mixed = []
    for sc in _mixed(p, scs, seed=17):
        h = synth.heterogeneous(rng, sc, p)
        mixed.append(dataclasses.replace(h, agent_q=_f32(h.agent_q), agent_r=_f32(h.agent_r),
                                         agent_lo=_f32(h.agent_lo), agent_hi=_f32(h.agent_hi)))
    K = 40
    kw = dict(alpha=1.6, state_box=True, s_lo=(-2.0, -2.0), s_hi=(2.0, 2.0), max_iter=K, eps_abs=0.0, eps_rel=0.0)
    g = gc.gpu_solve(p, mixed, solver_kw=kw)
    o = gc.oracle_same_instance(p, mixed, gc.oracle_opts(kw, lockstep=K), threads=4)
    for sc, gr, orr in zip(mixed, g, o):
        rel = gc.rel_traj_err(gr, orr)
        _say(f"  N={sc.N} T={sc.T}: rel {rel:.2e}")
        assert rel <= gc.REL_TOL
