"""Momentum ADMM (the fast ADMM with restart of Goldstein et al. 2014, Alg.
8, on the consensus block) on the device against the oracle's, through the
C ABI.  Lockstep runs follow the oracle's iterates (including its restart
decisions) to the parity bar; with frozen normals the momentum run converges
to the oracle's solution of the same QP; the three modes agree bitwise; the
option's limits are errors.
The derivative of a momentum solve is tested with the others
(tests/test_gpu_adjoint.py)."""
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

MOM = dict(momentum=True, mom_eta=0.999)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_momentum_lockstep_matches_oracle(cfg):
    p, scs = synth.config1() if cfg == "c1" else synth.config2(S=12)
    K = 40
    _say(f"momentum lockstep {cfg} K={K}")
    kw = dict(MOM, max_iter=K, eps_abs=0.0, eps_rel=0.0)
    g = gc.gpu_solve(p, scs, solver_kw=kw)
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(kw, lockstep=K), threads=4)
    plain = gc.gpu_solve(p, scs, solver_kw=dict(max_iter=K, eps_abs=0.0, eps_rel=0.0))
    worst, differs = 0.0, 0
    for sc, gr, orr, pr in zip(scs, g, o, plain):
        assert orr["iters"] == K and (gr["iters"] == K or (gr["status"] == tadmm.SCEN_CONVERGED and
                                                            gr["r_norm"] == 0.0 and gr["s_norm"] == 0.0))
        rel = gc.rel_traj_err(gr, orr)
        worst = max(worst, rel)
        assert rel <= gc.REL_TOL, (sc.N, sc.T, rel)
        differs += gc.rel_traj_err(pr, orr) > 10 * gc.REL_TOL
    _say(f"  worst rel {worst:.2e}; {differs} of {len(scs)} differ from plain ADMM beyond 10x the bar")
    assert differs >= max(1, len(scs) // 2)


def test_momentum_frozen_limit_matches_oracle():
    p = synth.ProblemParams(dp=2, u_max=2.0)
    T = 20
    sc = synth.Scenario(starts=np.array([[-3.0, 0.6], [3.0, -0.6]]), goals=np.array([[3.0, 0.1], [-3.0, -0.1]]), T=T)
    nrm = np.zeros((1, T, 2))
    nrm[..., 1] = 1.0
    base = dict(MOM, normal_mode=tadmm.NORMAL_FROZEN, rho=10.0)
    g = gc.gpu_solve(p, [sc], normals=[nrm], solver_kw=dict(base, max_iter=20000, eps_abs=1e-6, eps_rel=1e-6))[0]
    g1 = gc.gpu_solve(p, [sc], normals=[nrm], solver_kw=dict(normal_mode=tadmm.NORMAL_FROZEN, rho=10.0,
                                                             max_iter=20000, eps_abs=1e-6, eps_rel=1e-6))[0]
    o = gc.oracle_same_instance(p, [sc], gc.oracle_opts(dict(base, max_iter=20000, eps_abs=1e-11, eps_rel=1e-11)),
                                normals=[nrm])[0]
    rel = gc.rel_traj_err(g, o)
    _say(f"  iterations: momentum {g['iters']}, plain {g1['iters']}; rel {rel:.2e}")
    assert o["status"] == oracle.CONVERGED and g["status"] == tadmm.SCEN_CONVERGED
    assert rel <= gc.REL_TOL


def test_momentum_modes_bitwise_equal():
    """Plain (host loop, an extrapolation kernel after each test), batched
    (the persistent kernel's momentum variant) and many-workgroup (an
    extrapolation kernel in each captured iteration) agree bitwise."""
    p, scs = synth.config2(S=10)
    kw = dict(MOM, max_iter=100)
    a = gc.gpu_solve(p, scs, mode=tadmm.MODE_PLAIN, solver_kw=kw)
    for mode in (tadmm.MODE_BATCHED, tadmm.MODE_WIDE):
        b = gc.gpu_solve(p, scs, mode=mode, solver_kw=kw)
        for ga, gb in zip(a, b):
            assert ga["iters"] == gb["iters"] and ga["status"] == gb["status"]
            np.testing.assert_array_equal(ga["x"], gb["x"])


def test_momentum_limits_are_errors():
    p, scs = synth.config0()
    pk = synth.pack(p, scs)
    solver = tadmm.Solver(tadmm.make_params(p, max_iter=50, **MOM))
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag)
    with pytest.raises(tadmm.TadmmError) as e:
        prep.sqp(tadmm.MODE_BATCHED)
    assert "error 1" in str(e.value)
    prep.run(tadmm.MODE_BATCHED)
    prep.polish()     # the derivative of the converged point (tests/test_gpu_adjoint.py)
    solver.close()
