"""Heterogeneous agents (per-agent Q/R diagonals and input boxes) on the
device against the oracle, through the C ABI.  The per-agent arrays are
rounded to FP32 on the host, so both sides solve the instance the device
receives."""
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


def _hetero(S=12, seed=7):
    p, scs = synth.config2(S=S)
    rng = np.random.default_rng(seed)
    out = []
    for sc in scs:
        h = synth.heterogeneous(rng, sc, p)
        out.append(dataclasses.replace(h, agent_q=_f32(h.agent_q), agent_r=_f32(h.agent_r),
                                       agent_lo=_f32(h.agent_lo), agent_hi=_f32(h.agent_hi)))
    return p, out


def test_hetero_lockstep_matches_oracle():
    p, scs = _hetero()
    K = 40
    _say(f"heterogeneous lockstep K={K}, N = {[s.N for s in scs]}")
    g = gc.gpu_solve(p, scs, solver_kw=dict(max_iter=K, eps_abs=0.0, eps_rel=0.0))
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(lockstep=K))
    worst = 0.0
    for sc, gr, orr in zip(scs, g, o):
        assert gr["iters"] == K or (gr["status"] == tadmm.SCEN_CONVERGED and gr["r_norm"] == 0.0
                                    and gr["s_norm"] == 0.0)
        rel = gc.rel_traj_err(gr, orr)
        worst = max(worst, rel)
        assert rel <= gc.REL_TOL, (sc.N, sc.T, rel)
        # every agent within its own box
        assert np.all(gr["u"] <= sc.agent_hi[:, None, :] + 1e-6) and np.all(gr["u"] >= sc.agent_lo[:, None, :] - 1e-6)
    _say(f"  worst rel {worst:.2e}")


def test_hetero_converged_solves_match_oracle():
    p, scs = _hetero(S=24, seed=11)
    g = gc.gpu_solve(p, scs)
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts())
    n = 0
    for sc, gr, orr in zip(scs, g, o):
        if orr["status"] != oracle.CONVERGED:
            continue
        n += 1
        assert gr["status"] == tadmm.SCEN_CONVERGED, (sc.N, sc.T)
        rel = gc.rel_traj_err(gr, orr)
        assert rel <= gc.REL_TOL, (sc.N, sc.T, rel)
    _say(f"  {n} converged scenarios compared")
    assert n >= 3


def test_hetero_modes_bitwise_equal():
    p, scs = _hetero(S=10, seed=3)
    kw = dict(max_iter=100)
    a = gc.gpu_solve(p, scs, mode=tadmm.MODE_PLAIN, solver_kw=kw)
    for mode in (tadmm.MODE_BATCHED, tadmm.MODE_WIDE):
        b = gc.gpu_solve(p, scs, mode=mode, solver_kw=kw)
        for ga, gb in zip(a, b):
            assert ga["iters"] == gb["iters"]
            np.testing.assert_array_equal(ga["x"], gb["x"])


def test_hetero_bad_inputs_and_derivative_rejected():
    p, scs = _hetero(S=2, seed=5)
    pk = synth.pack(p, scs)
    solver = tadmm.Solver(tadmm.make_params(p))
    bad_q = pk.agent_q.copy()
    bad_q[1, 0] = -1.0
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag, agent_q=bad_q)
    with pytest.raises(tadmm.TadmmError) as e:
        prep.run(tadmm.MODE_BATCHED)
    assert "error 3" in str(e.value)
    lo = pk.agent_lo.copy()
    lo[0, 1] = pk.agent_hi[0, 1]
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag, agent_lo=lo,
                          agent_hi=pk.agent_hi)
    with pytest.raises(tadmm.TadmmError) as e:
        prep.run(tadmm.MODE_BATCHED)
    assert "error 3" in str(e.value)
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag, agent_lo=pk.agent_lo)
    with pytest.raises(tadmm.TadmmError) as e:
        prep.run(tadmm.MODE_BATCHED)
    assert "error 1" in str(e.value)
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag, agent_q=pk.agent_q,
                          agent_r=pk.agent_r, agent_lo=pk.agent_lo, agent_hi=pk.agent_hi)
    prep.run(tadmm.MODE_BATCHED)
    with pytest.raises(tadmm.TadmmError) as e:
        prep.polish()
    assert "error 1" in str(e.value)
    solver.close()
