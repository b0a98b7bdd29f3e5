"""The options in 3-D (nx = 6, nu = 3: the per-axis split with three axes,
and the one-lane-per-agent path): over-relaxation, momentum, the state
boxes, adaptive penalties and per-agent dynamics, each in lockstep with the
oracle on small 3-D crossings, and the three modes bitwise equal."""
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
    "boxes": dict(state_box=True, s_lo=(-2.0,) * 3, s_hi=(2.0,) * 3, p_lo=(-4.9,) * 3, p_hi=(4.9,) * 3),
    "adaptive": dict(adaptive_rho=True, rho_mu=10.0, rho_tau=2.0, rho_every=1),
    "dynamics": {},
}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _crossings(with_dynamics):
    p = synth.ProblemParams(dp=3, u_max=3.0)
    _, base = synth.config2(S=40)
    base = [s for s in base if s.N <= 10][:4]
    rng = np.random.default_rng(6)
    scs = [synth.Scenario(starts=np.concatenate([s.starts, rng.uniform(-4.5, 4.5, (s.N, 1))], 1),
                          goals=np.concatenate([s.goals, rng.uniform(-4.5, 4.5, (s.N, 1))], 1), T=s.T) for s in base]
    if with_dynamics:
        f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
        scs = [dataclasses.replace(m, agent_A=f32(m.agent_A), agent_B=f32(m.agent_B))
               for m in (synth.mixed_dynamics(rng, sc, p) for sc in scs)]
    return p, scs


@pytest.mark.parametrize("name", sorted(OPTIONS))
def test_option_3d_lockstep_matches_oracle(name):
    p, scs = _crossings(name == "dynamics")
    K = 30
    kw = dict(OPTIONS[name], max_iter=K, eps_abs=0.0, eps_rel=0.0)
    g = gc.gpu_solve(p, scs, solver_kw=kw)
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(kw, lockstep=K), threads=4)
    worst = 0.0
    for sc, gr, orr in zip(scs, g, o):
        rel = gc.rel_traj_err(gr, orr)
        worst = max(worst, rel)
        assert rel <= gc.REL_TOL, (name, sc.N, sc.T, rel)
    _say(f"  3-D {name}: N = {[s.N for s in scs]}, worst rel {worst:.2e}")


@pytest.mark.parametrize("name", ["relaxed", "momentum", "boxes"])
def test_option_3d_modes_bitwise_equal(name):
    p, scs = _crossings(False)
    kw = dict(OPTIONS[name], max_iter=60)
    a = gc.gpu_solve(p, scs, mode=tadmm.MODE_PLAIN, solver_kw=kw)
    for mode in (tadmm.MODE_BATCHED, tadmm.MODE_WIDE):
        b = gc.gpu_solve(p, scs, mode=mode, solver_kw=kw)
        for ga, gb in zip(a, b):
            assert ga["iters"] == gb["iters"]
            np.testing.assert_array_equal(ga["x"], gb["x"])
