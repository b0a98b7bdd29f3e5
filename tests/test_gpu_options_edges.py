"""Edge cases of the options (over-relaxation, momentum, state boxes,
per-agent dynamics): a tiny mixed batch with a single agent, a horizon of
one step and a three-agent swap, in lockstep with the oracle; and the empty
batch, which every option accepts as a no-op."""
import dataclasses
import sys

import numpy as np
import pytest

import synth
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_15838_amd as tadmm  # noqa: E402

OPTIONS = {
    "relaxed": dict(alpha=1.6),
    "momentum": dict(momentum=True),
    "boxes": dict(state_box=True, s_lo=(-1.5, -1.5), s_hi=(1.5, 1.5), p_lo=(-0.2, -0.2), p_hi=(1.7, 1.7)),
    "dynamics": {},
}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _tiny(with_dynamics):
    scs = [synth.Scenario(starts=np.array([[0.0, 0.0], [1.0, 0.0]]), goals=np.array([[1.0, 0.0], [0.0, 0.0]]), T=1),
           synth.Scenario(starts=np.array([[0.0, 0.0]]), goals=np.array([[1.0, 1.0]]), T=3),
           synth.Scenario(starts=np.array([[0.0, 0.0], [0.0, 1.5], [1.5, 0.0]]),
                          goals=np.array([[1.5, 1.5], [1.5, 0.0], [0.0, 1.5]]), T=7)]
    if with_dynamics:
        p = synth.ProblemParams(dp=2)
        rng = np.random.default_rng(4)
        f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
        scs = [dataclasses.replace(m, agent_A=f32(m.agent_A), agent_B=f32(m.agent_B))
               for m in (synth.mixed_dynamics(rng, sc, p) for sc in scs)]
    return scs


@pytest.mark.parametrize("name", sorted(OPTIONS))
def test_tiny_mixed_batch_lockstep(name):
    p = synth.ProblemParams(dp=2)
    scs = _tiny(name == "dynamics")
    K = 25
    kw = dict(OPTIONS[name], max_iter=K, eps_abs=0.0, eps_rel=0.0)
    g = gc.gpu_solve(p, scs, solver_kw=kw)
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(kw, lockstep=K))
    for sc, gr, orr in zip(scs, g, o):
        rel = gc.rel_traj_err(gr, orr)
        _say(f"  {name}: N={sc.N} T={sc.T}: iterations {gr['iters']}, rel {rel:.2e}")
        assert rel <= gc.REL_TOL
        assert gr["iters"] == K or (gr["status"] == tadmm.SCEN_CONVERGED and gr["r_norm"] == 0.0
                                    and gr["s_norm"] == 0.0)


@pytest.mark.parametrize("name", sorted(OPTIONS))
def test_empty_batch_with_option(name):
    p = synth.ProblemParams(dp=2)
    solver = tadmm.Solver(tadmm.make_params(p, **OPTIONS[name]))
    z = lambda *s: np.zeros(s)
    extra = dict(agent_A=z(0, 16), agent_B=z(0, 8)) if name == "dynamics" else {}
    prep = solver.prepare(np.zeros(0, np.int32), np.zeros(0, np.int32), z(0, 4), z(0, 4), z(0, 4), z(0, 2),
                          **extra)
    prep.run(tadmm.MODE_BATCHED)
    solver.close()
