"""The SQP outer loop on the device (tadmm_sqp) against the oracle's
(oracle/sqp.py): half-planes re-linearized about each round's solution, the
stopping rule of Sec. V-A.  Bar: the same number of rounds and outcome, the
objective within 1e-5 relative, the solution within the parity bar (1e-4
relative trajectory error), on the FP32 instance the device receives.  The
device continues each round from the previous one (warm start); the oracle
starts every round from the references.  Each round's QP has one
minimiser, and each side stops within its ADMM tolerance of it; where that
minimiser is ill-conditioned (a nearly flat direction along touching
constraints), or the loop ends at max_rounds short of a fixed point, the
tolerance allows more than that, and the bars (trajectory, objective,
smallest distance) are 10 times the oracle's own distance between its
results at tolerances 1e-6 and 1e-8 (the principle of the bar of capped
runs).  After a round that did not converge, the device restarts the duals
(the oracle always does), so an infeasible first linearization costs both
sides the same."""
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


def _device_sqp(p, scs, mode, **kw):
    pk = synth.pack(p, scs)
    solver = tadmm.Solver(tadmm.make_params(p, **KW))
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag)
    st = prep.sqp(mode, **kw).cpu().numpy()
    res = tadmm.split_outputs(prep.result(), pk.n_agents, pk.horizon, p.nx, p.nu)
    return res, st, prep, solver


_ORACLE = {}   # the oracle's results, shared by the modes' tests


def _oracle_sqp(p, scs, eps=KW["eps_abs"], max_iter=KW["max_iter"], **kw):
    key = (id(p), tuple(id(sc) for sc in scs), eps, max_iter, tuple(sorted(kw.items())))
    if key not in _ORACLE:
        o = oracle.OracleOptions(max_iter=max_iter, eps_abs=eps, eps_rel=eps)
        _ORACLE[key] = osqp.sqp_solve(gc.Fp32Problem(p), scs, o, inputs=[gc.fp32_inputs(sc) for sc in scs], **kw)
    return _ORACLE[key]


_CASES = None


def _cases():
    global _CASES
    if _CASES is None:
        p0, s0 = synth.config0()
        p2, s2 = synth.config2(S=40)
        _CASES = [(p0, s0), (p2, [s for s in s2 if s.N <= 8][:6])]
    return _CASES


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_sqp_matches_oracle(mode):
    for p, scs in _cases():
        _say(f"SQP mode {mode}: {len(scs)} scenarios, N = {[s.N for s in scs]}")
        res, st, _, solver = _device_sqp(p, scs, mode, max_rounds=10)
        solver.close()
        ref = _oracle_sqp(p, scs, max_rounds=10)
        for k, (g, r) in enumerate(zip(res, ref)):
            rounds, conv, J, ms = st[k]
            Jr, msr = r["objective"][-1], r["min_sep"][-1]
            rel, jrel, dms = gc.rel_traj_err(g, r), abs(J - Jr) / abs(Jr), abs(ms - msr)
            bar, jbar, msbar = gc.REL_TOL, 1e-5, 1e-4
            if rel > bar or jrel > jbar or dms > msbar:   # the oracle's own distance from its tight solution
                tight = _oracle_sqp(p, [scs[k]], eps=1e-8, max_iter=40000, max_rounds=r["rounds"], rtol=0.0)[0]
                bar = max(bar, 10.0 * gc.rel_traj_err(dict(x=r["x"], u=r["u"]), tight))
                jbar = max(jbar, 10.0 * abs(Jr - tight["objective"][-1]) / abs(Jr))
                msbar = max(msbar, 10.0 * abs(msr - tight["min_sep"][-1]))
            _say(f"  scenario {k}: rounds {int(rounds)} / {r['rounds']}, converged {bool(conv)} / {r['converged']}, "
                 f"J {J:.6f} / {Jr:.6f} (bar {jbar:.1e}), rel {rel:.2e} (bar {bar:.1e}), last-round iterations "
                 f"{g['iters']} (warm) / {r['iters']} (cold)")
            assert int(rounds) == r["rounds"] and bool(conv) == r["converged"]
            assert jrel <= jbar and rel <= bar and dms <= msbar


def test_sqp_modes_bitwise_equal():
    p, scs = _cases()[1]
    outs = [_device_sqp(p, scs, mode, max_rounds=10) for mode in (0, 1, 2)]
    for res, st, _, solver in outs[1:]:
        np.testing.assert_array_equal(st, outs[0][1])
        for a, b in zip(res, outs[0][0]):
            np.testing.assert_array_equal(a["x"], b["x"])
            np.testing.assert_array_equal(a["u"], b["u"])
    for *_, solver in outs:
        solver.close()


def test_sqp_one_round_is_a_frozen_normal_solve():
    """max_rounds = 1 is one solve with the reference normals frozen."""
    p, scs = _cases()[1]
    res, st, _, solver = _device_sqp(p, scs, tadmm.MODE_BATCHED, max_rounds=1)
    solver.close()
    ref = gc.gpu_solve(p, scs, solver_kw=dict(KW, normal_mode=tadmm.NORMAL_FROZEN))
    for a, b in zip(res, ref):
        np.testing.assert_array_equal(a["x"], b["x"])
        assert a["iters"] == b["iters"]
    assert np.all(st[:, 0] == 1) and np.all(st[:, 1] == 0)


def test_sqp_argument_and_state_errors():
    p, scs = _cases()[0]
    res, st, prep, solver = _device_sqp(p, scs, tadmm.MODE_BATCHED, max_rounds=3)
    with pytest.raises(tadmm.TadmmError) as e:
        prep.polish()             # the derivative is defined for tadmm_solve results
    assert "error 7" in str(e.value)
    for bad in (dict(max_rounds=0), dict(rtol=-1.0), dict(sep_tol=float("nan"))):
        with pytest.raises(tadmm.TadmmError) as e:
            prep.sqp(tadmm.MODE_BATCHED, **bad)
        assert "error 1" in str(e.value)
    with pytest.raises(tadmm.TadmmError):
        prep.sqp(7)
    solver.close()
