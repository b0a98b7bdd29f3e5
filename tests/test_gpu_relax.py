"""Over-relaxed ADMM (Boyd et al. 2011, Sec. 3.4.3: the consensus and dual
updates take alpha C x^(k+1) + (1 - alpha) z^k) on the device against the
oracle's, through the C ABI.  Lockstep runs follow the oracle's iterates to
the parity bar; with frozen normals the relaxed run converges to the oracle's
solution of the same QP in fewer iterations than plain ADMM; the three modes
agree bitwise; SQP rounds (whose restarts reset the copies' z) match the
oracle's.  The derivative of a relaxed solve is tested with the others
(tests/test_gpu_adjoint.py)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import sqp as osqp
from tests import gpu_common as gc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2602_15838_amd as tadmm  # noqa: E402

ALPHA = 1.6


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("cfg, alpha", [("c1", ALPHA), ("c2", ALPHA), ("c2", 0.7)])
def test_relaxed_lockstep_matches_oracle(cfg, alpha):
    p, scs = synth.config1() if cfg == "c1" else synth.config2(S=12)
    K = 40
    _say(f"relaxed lockstep {cfg} alpha={alpha} K={K}")
    kw = dict(alpha=alpha, max_iter=K, eps_abs=0.0, eps_rel=0.0)
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
    assert differs >= max(1, len(scs) // 2)       # relaxation changes the iterates


def _side_pass(T=20):
    sc = synth.Scenario(starts=np.array([[-3.0, 0.6], [3.0, -0.6]]), goals=np.array([[3.0, 0.1], [-3.0, -0.1]]), T=T)
    nrm = np.zeros((1, T, 2))
    nrm[..., 1] = 1.0
    return sc, nrm


def test_relaxed_frozen_limit_matches_oracle_in_fewer_iterations():
    p = synth.ProblemParams(dp=2, u_max=2.0)
    sc, nrm = _side_pass()
    base = dict(normal_mode=tadmm.NORMAL_FROZEN, rho=10.0)
    run = dict(base, max_iter=20000, eps_abs=1e-6, eps_rel=1e-6)
    g = gc.gpu_solve(p, [sc], normals=[nrm], solver_kw=dict(run, alpha=ALPHA))[0]
    g1 = gc.gpu_solve(p, [sc], normals=[nrm], solver_kw=run)[0]
    o = gc.oracle_same_instance(p, [sc], gc.oracle_opts(dict(base, alpha=ALPHA, max_iter=20000, eps_abs=1e-11,
                                                             eps_rel=1e-11)), normals=[nrm])[0]
    rel = gc.rel_traj_err(g, o)
    _say(f"  iterations: alpha {ALPHA} {g['iters']}, plain {g1['iters']}; rel {rel:.2e}")
    assert o["status"] == oracle.CONVERGED and g["status"] == tadmm.SCEN_CONVERGED
    assert rel <= gc.REL_TOL
    assert g["iters"] < g1["iters"]


def test_relaxed_modes_bitwise_equal():
    p, scs = synth.config2(S=10)
    kw = dict(alpha=ALPHA, max_iter=100)
    a = gc.gpu_solve(p, scs, mode=tadmm.MODE_PLAIN, solver_kw=kw)
    for mode in (tadmm.MODE_BATCHED, tadmm.MODE_WIDE):
        b = gc.gpu_solve(p, scs, mode=mode, solver_kw=kw)
        for ga, gb in zip(a, b):
            assert ga["iters"] == gb["iters"] and ga["status"] == gb["status"]
            np.testing.assert_array_equal(ga["x"], gb["x"])


def test_relaxed_with_adaptive_rho_and_box_lockstep():
    """All three options together in lockstep with the oracle."""
    p, scs = synth.config2(S=6)
    K = 40
    kw = dict(alpha=ALPHA, adaptive_rho=True, rho_mu=10.0, rho_tau=2.0, rho_every=1, state_box=True,
              s_lo=(-2.0, -2.0), s_hi=(2.0, 2.0), max_iter=K, eps_abs=0.0, eps_rel=0.0)
    g = gc.gpu_solve(p, scs, solver_kw=kw)
    o = gc.oracle_same_instance(p, scs, gc.oracle_opts(kw, lockstep=K), threads=4)
    for sc, gr, orr in zip(scs, g, o):
        rel = gc.rel_traj_err(gr, orr)
        _say(f"  N={sc.N} T={sc.T}: rel {rel:.2e}")
        assert rel <= gc.REL_TOL


def test_relaxed_sqp_matches_oracle():
    """Config 0 through the SQP loop with alpha = 1.6: the same rounds and
    outcome as the oracle's loop, the solution within the parity bar."""
    p, scs = synth.config0()
    KW = dict(max_iter=5000, eps_abs=1e-6, eps_rel=1e-6)
    pk = synth.pack(p, scs)
    solver = tadmm.Solver(tadmm.make_params(p, alpha=ALPHA, **KW))
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag)
    st = prep.sqp(tadmm.MODE_BATCHED, max_rounds=10).cpu().numpy()
    res = tadmm.split_outputs(prep.result(), pk.n_agents, pk.horizon, p.nx, p.nu)
    with pytest.raises(tadmm.TadmmError):
        prep.polish()             # the derivative is defined for tadmm_solve results
    solver.close()
    o = oracle.OracleOptions(alpha=float(np.float32(ALPHA)), **KW)
    ref = osqp.sqp_solve(gc.Fp32Problem(p), scs, o, inputs=[gc.fp32_inputs(sc) for sc in scs], max_rounds=10)
    for k, (g, r) in enumerate(zip(res, ref)):
        rounds, conv, J, ms = st[k]
        rel = gc.rel_traj_err(g, r)
        _say(f"  rounds {int(rounds)} / {r['rounds']}, J {J:.6f} / {r['objective'][-1]:.6f}, rel {rel:.2e}")
        assert int(rounds) == r["rounds"] and bool(conv) == r["converged"]
        assert rel <= gc.REL_TOL
        assert abs(J - r["objective"][-1]) <= 1e-5 * abs(r["objective"][-1])


