"""The ablation variants' work ordering (Sec. V-B, Table II) and the
agent-count sweep, through the C-ABI library."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2602_15838_amd import study  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_ablation_ordering_and_same_iterates():
    """Base >= Hotstart >= Turbo in active-set passes at every agent count,
    Base rebuilds the most factors, and all three reach the same iterates."""
    agents = (2, 6, 14)
    recs = study.ablation(seeds=4, agents=agents)
    by = {(r["agents"], r["variant"]): r for r in recs}
    for N in agents:
        b, h, t = (by[(N, v)] for v in ("base", "hotstart", "turbo"))
        _say(f"N={N}: passes base {b['active_set_passes']} hotstart {h['active_set_passes']} "
               f"turbo {t['active_set_passes']}; iters {b['admm_iters']}/{h['admm_iters']}/{t['admm_iters']}")
        assert b["active_set_passes"] >= h["active_set_passes"] >= t["active_set_passes"], N
        assert b["refactored_stages"] >= h["refactored_stages"], N
        # the same iterates: the same iteration counts and outcomes
        assert b["admm_iters"] == h["admm_iters"] == t["admm_iters"], N
        assert b["converged"] == h["converged"] == t["converged"], N
        for r in (b, h):
            assert r["max_rel_state_diff_vs_turbo"] <= 1e-4, (N, r)


def test_sweep_small():
    """The sweep's records: every solve ends normally (the symmetric sphere
    swaps run to the iteration cap), both paths time it, and the fit record
    holds finite exponents."""
    recs = study.sweep(agents=(2, 4, 8))
    rows = [r for r in recs if r["study"] == "sweep"]
    assert [r["agents"] for r in rows] == [2, 4, 8]
    for r in rows:
        assert r["status"] in (0, 1) and r["plain_ms_per_solve"] > 0 and r["wide_ms_per_solve"] > 0
    fit = recs[-1]
    assert fit["study"] == "sweep_fit" and np.isfinite(fit["plain_time_exponent"])


@pytest.mark.parametrize("variant", ["base", "hotstart", "turbo"])
def test_ablation_variant_lockstep_with_oracle(variant):
    """Each ablation variant (the start strategies of Sec. V-B: Base,
    Hotstart, Turbo) against the oracle run with the same strategy (start of
    every local QP, hotstart, factor reuse): 25 iterations in lockstep on
    three 6-agent crossings of the study, trajectories, working sets,
    active half-planes and every iteration's residual norms.  The work
    counts of both sides are printed; each side's Base needs the most
    active-set passes."""
    from tests import gpu_common as gc
    flags = study.VARIANTS[variant]
    p, scs = study.ablation_scenarios(6, 3)
    K = 25
    kw = dict(flags, eps_abs=0.0, eps_rel=0.0, max_iter=K)
    _say(f"ablation variant {variant} lockstep K={K}")
    g = gc.gpu_solve(p, scs, solver_kw=kw, history=True)
    opts = gc.oracle_opts(kw, lockstep=K)
    opts.lu_reuse = bool(flags["cache_factors"])
    o = gc.oracle_same_instance(p, scs, opts, keep_zl=True)
    worst = 0.0
    for sc, gr, orr in zip(scs, g, o):
        assert gr["iters"] == K and orr["iters"] == K
        rep = gc.compare(p, sc, gr, orr)
        gc.compare_history(gr, orr, sc, p.dp)
        worst = max(worst, rep["rel"])
    gp = [int(gr["counters"][0]) for gr in g]
    op = [int(orr["as_passes"]) for orr in o]
    _say(f"  worst rel {worst:.2e}; active-set passes device (axis problems) {gp}, oracle (agent QPs) {op}")
    if variant == "base":
        base = study.VARIANTS["turbo"]
        t = gc.gpu_solve(p, scs, solver_kw=dict(base, eps_abs=0.0, eps_rel=0.0, max_iter=K))
        to = gc.oracle_same_instance(p, scs, gc.oracle_opts(dict(base, max_iter=K), lockstep=K))
        assert sum(gp) > sum(int(x["counters"][0]) for x in t)
        assert sum(op) > sum(int(x["as_passes"]) for x in to)
