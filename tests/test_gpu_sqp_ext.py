"""The SQP outer loop (tadmm_sqp) with the extensions: a velocity box,
heterogeneous agents (per-agent weights in the objective of the stopping
rule), adaptive penalties and per-agent dynamics, against the oracle's loop (oracle/sqp.py) on the FP32 instance the
device receives.  The bars are those of the plain loop's test: the same
rounds and outcome, the objective within 1e-5 relative, the trajectories
within the parity bar, or within 10 times the oracle's own distance between
its results at ADMM tolerances 1e-6 and 1e-8 where that is larger."""
import dataclasses
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

KW = dict(max_iter=5000, eps_abs=1e-6, eps_rel=1e-6)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _compare(p, scs, extra):
    pk = synth.pack(p, scs)
    solver = tadmm.Solver(tadmm.make_params(p, **KW, **extra))
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag, agent_q=pk.agent_q,
                          agent_r=pk.agent_r, agent_lo=pk.agent_lo, agent_hi=pk.agent_hi, agent_A=pk.agent_A,
                          agent_B=pk.agent_B)
    st = prep.sqp(tadmm.MODE_BATCHED, max_rounds=10).cpu().numpy()
    res = tadmm.split_outputs(prep.result(), pk.n_agents, pk.horizon, p.nx, p.nu)
    solver.close()

    def ref(scs_, eps, max_iter, **kw):
        o = gc.oracle_opts(dict(extra, max_iter=max_iter, eps_abs=eps, eps_rel=eps))
        return osqp.sqp_solve(gc.Fp32Problem(p), scs_, o, inputs=[gc.fp32_inputs(sc) for sc in scs_],
                              max_rounds=10, **kw)

    out = ref(scs, KW["eps_abs"], KW["max_iter"])
    for k, (g, r) in enumerate(zip(res, out)):
        rounds, conv, J, ms = st[k]
        Jr = r["objective"][-1]
        rel, jrel = gc.rel_traj_err(g, r), abs(J - Jr) / abs(Jr)
        bar, jbar = gc.REL_TOL, 1e-5
        if rel > bar or jrel > jbar:
            tight = ref([scs[k]], 1e-8, 40000, rtol=0.0)[0]
            bar = max(bar, 10.0 * gc.rel_traj_err(dict(x=r["x"], u=r["u"]), tight))
            jbar = max(jbar, 10.0 * abs(Jr - tight["objective"][-1]) / abs(Jr))
        _say(f"  scenario {k} (N={scs[k].N}): rounds {int(rounds)} / {r['rounds']}, converged {bool(conv)} / "
             f"{r['converged']}, J {J:.6f} / {Jr:.6f}, rel {rel:.2e} (bar {bar:.1e})")
        assert int(rounds) == r["rounds"] and bool(conv) == r["converged"]
        assert jrel <= jbar and rel <= bar
    return res


def test_sqp_with_velocity_box_matches_oracle():
    p, scs = synth.config0()
    extra = dict(state_box=True, s_lo=(-2.5, -2.5), s_hi=(2.5, 2.5))
    res = _compare(p, scs, extra)
    for g in res:
        assert np.abs(g["x"][:, 1:, p.dp:]).max() <= 2.5 + 1e-3


def test_sqp_with_heterogeneous_agents_matches_oracle():
    p, s2 = synth.config2(S=40)
    rng = np.random.default_rng(13)
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    scs = []
    for sc in [s for s in s2 if s.N <= 8][:4]:
        h = synth.heterogeneous(rng, sc, p)
        scs.append(dataclasses.replace(h, agent_q=f32(h.agent_q), agent_r=f32(h.agent_r), agent_lo=f32(h.agent_lo),
                                       agent_hi=f32(h.agent_hi)))
    _compare(p, scs, {})


def test_sqp_with_adaptive_rho_matches_oracle():
    """Residual balancing inside the rounds: the device's rounds continue with
    the adapted penalty, the oracle's restart from the initial one; each
    round's QP has one minimiser, so the bars are the same."""
    p, scs = synth.config0()
    _compare(p, scs, dict(adaptive_rho=True, rho_mu=10.0, rho_tau=2.0, rho_every=1))


def test_sqp_with_agent_dynamics_matches_oracle():
    p, s2 = synth.config2(S=40)
    rng = np.random.default_rng(17)
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    scs = [dataclasses.replace(m, agent_A=f32(m.agent_A), agent_B=f32(m.agent_B))
           for m in (synth.mixed_dynamics(rng, sc, p) for sc in [s for s in s2 if s.N <= 8][:3])]
    _compare(p, scs, {})
