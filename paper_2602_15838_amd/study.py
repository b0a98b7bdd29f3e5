"""Work counts of the solver's ablation variants, and an agent-count sweep.

Ablation (Sec. V-B, Table II).  The paper compares three ADMM variants that
differ only in how each local QP is started: a cold-started active-set
solver (BaseADMM), the parametric hotstart alone (HotstartADMM), and the
Riccati warm start of the first iteration plus the hotstart (TurboADMM).
Here the same three are switches of the solver:

  base      every local QP starts from u = 0 and an empty working set, and
            the Riccati factors are rebuilt on every active-set pass;
  hotstart  iteration k >= 2 starts from the previous iterate and working
            set, and the factors are kept while the working set is
            unchanged (the analogue of reusing the QP factorization);
            iteration 1 starts from u = 0;
  turbo     hotstart plus the warm start of iteration 1 from the
            unconstrained Riccati solution, clipped to the input box
            (Sec. IV-B).

Every local QP has a unique minimiser, so the three variants run the same
ADMM iterates up to rounding; what changes is the number of active-set
passes (the counterpart of the paper's QP iterations), of refactored
agent-stages, and the time.  The scenarios are crossings at the paper's
agent counts (2, 4, 6, 10, 14; T = 20): starts and goals drawn in a 10 x 10
box at least 1 apart, joined by straight-line references, 20 seeds each, as
its timings are averages over 20 runs.

Sweep (Sec. V-C, the scaling claim).  Time per ADMM iteration against the
agent count for one 3-D sphere swap per N (T = 50, the radius grown as
sqrt(N) so that the density of agents on the sphere stays that of 128 agents
at radius 12), through the plain path and the many-workgroup path, with the
least-squares exponent of time against N.  The swaps are symmetric and run
to the 200-iteration cap, so the iteration count is fixed and the per-solve
times scale as the per-iteration ones.

SQP (the outer re-linearization loop, tadmm_sqp).  The benchmark's ragged
batch (4096 scenarios) through the SQP loop in the batched mode, with the
stopping rule of Sec. V-A (relative objective change 1e-4, every pair at
least d_min - sep_tol apart): wall time, rounds, outcomes, and the same
batch through one solve with the normals re-linearized every iteration.

Penalty (adaptive rho).  The benchmark's batch with rho fixed and adapted
by residual balancing: converged fraction, iterations, refactors, time.

    python -m paper_2602_15838_amd.study [--ablation] [--sweep] [--sqp] [--rho] [--seeds 20]

prints one JSON object per line.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from typing import Dict, List, Sequence

import numpy as np

VARIANTS = {
    "base": dict(cache_factors=False, riccati_warmstart=False, hotstart=False),
    "hotstart": dict(cache_factors=True, riccati_warmstart=False, hotstart=True),
    "turbo": dict(cache_factors=True, riccati_warmstart=True, hotstart=True),
}
ABLATION_AGENTS = (2, 4, 6, 10, 14)
SWEEP_AGENTS = (2, 4, 8, 16, 32, 64, 128)
STUDY_CONFIG_ID = 5          # seed stream of the study's scenarios


def fit_exponent(n: Sequence[float], y: Sequence[float]) -> float:
    """Least-squares slope of log y against log n (y ~ c n^e)."""
    ln, ly = np.log(np.asarray(n, np.float64)), np.log(np.asarray(y, np.float64))
    A = np.stack([ln, np.ones_like(ln)], axis=1)
    return float(np.linalg.lstsq(A, ly, rcond=None)[0][0])


def ablation_scenarios(N: int, seeds: int):
    import synth
    p = synth.ProblemParams(dp=2, u_max=2.0)
    scs = [synth.random_box(synth.rng_for(STUDY_CONFIG_ID, 1000 * N + s), N, 20) for s in range(seeds)]
    return p, scs


def sweep_scenario(N: int):
    import synth
    p = synth.ProblemParams(dp=3, u_max=3.0)
    return p, synth.sphere_swap(N, 12.0 * math.sqrt(N / 128.0), 50)


def _solve_one(solver, problem, sc, mode: int):
    """One scenario, solved twice (the second run timed).  Returns
    (seconds, result dict on the host)."""
    import torch

    import synth
    import paper_2602_15838_amd as tadmm
    pk = synth.pack(problem, [sc])
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag)
    prep.run(mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prep.run(mode)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = prep.result()
    out = dict(iters=int(r["iters"][0]), status=int(r["status"][0]), counters=r["counters"][0].cpu().numpy(),
               x=r["x"].cpu().numpy().astype(np.float64))
    del prep
    return dt, out


def ablation(seeds: int = 20, agents: Sequence[int] = ABLATION_AGENTS, mode: int = 0) -> List[Dict]:
    """One record per (agent count, variant): ADMM iterations, converged
    fraction, active-set passes and refactored agent-stages per solve (mean
    and standard deviation over the seeds), and milliseconds per solve; plus
    the largest trajectory difference of each variant from turbo's."""
    import paper_2602_15838_amd as tadmm
    recs = []
    for N in agents:
        problem, scs = ablation_scenarios(N, seeds)
        runs = {}
        for name, flags in VARIANTS.items():
            solver = tadmm.Solver(tadmm.make_params(problem, **flags))
            runs[name] = [_solve_one(solver, problem, sc, mode) for sc in scs]
            solver.close()
        for name in VARIANTS:
            rs = runs[name]
            passes = np.array([r["counters"][0] for _, r in rs], np.float64)
            refac = np.array([r["counters"][1] for _, r in rs], np.float64)
            ms = np.array([1e3 * dt for dt, _ in rs])
            dx = max(float(np.max(np.abs(r["x"] - t["x"])) / max(np.max(np.abs(t["x"])), 1e-30))
                     for (_, r), (_, t) in zip(rs, runs["turbo"]))
            recs.append(dict(study="ablation", agents=N, variant=name, seeds=len(rs),
                             admm_iters=round(float(np.mean([r["iters"] for _, r in rs])), 2),
                             converged=round(float(np.mean([r["status"] == tadmm.SCEN_CONVERGED for _, r in rs])), 3),
                             active_set_passes=round(float(passes.mean()), 1),
                             active_set_passes_std=round(float(passes.std()), 1),
                             refactored_stages=round(float(refac.mean()), 1),
                             ms_per_solve=round(float(ms.mean()), 3), ms_std=round(float(ms.std()), 3),
                             max_rel_state_diff_vs_turbo=float(f"{dx:.3e}")))
    return recs


def sweep(agents: Sequence[int] = SWEEP_AGENTS) -> List[Dict]:
    """One record per agent count (plain and many-workgroup times), then one
    record with the fitted exponents."""
    import paper_2602_15838_amd as tadmm
    recs = []
    for N in agents:
        problem, sc = sweep_scenario(N)
        solver = tadmm.Solver(tadmm.make_params(problem))
        rec = dict(study="sweep", agents=N, horizon=50, pair_steps=N * (N - 1) // 2 * 50)
        for name, mode in (("plain", tadmm.MODE_PLAIN), ("wide", tadmm.MODE_WIDE)):
            dt, r = _solve_one(solver, problem, sc, mode)
            rec[f"{name}_ms_per_solve"] = round(1e3 * dt, 3)
            rec[f"{name}_ms_per_iteration"] = round(1e3 * dt / max(r["iters"], 1), 4)
            rec["iters"], rec["status"] = r["iters"], r["status"]
        solver.close()
        recs.append(rec)
    ns = [r["agents"] for r in recs]
    fit = dict(study="sweep_fit", agents=list(ns))
    for name in ("plain", "wide"):
        fit[f"{name}_time_exponent"] = round(fit_exponent(ns, [r[f"{name}_ms_per_solve"] for r in recs]), 3)
        fit[f"{name}_per_iteration_exponent"] = round(
            fit_exponent(ns, [r[f"{name}_ms_per_iteration"] for r in recs]), 3)
    recs.append(fit)
    return recs


def sqp_study(S: int = 4096, max_rounds: int = 10, rtol: float = 1e-4, sep_tol: float = 1e-2) -> List[Dict]:
    import torch

    import synth
    import paper_2602_15838_amd as tadmm
    problem, scs = synth.config2(S=S)
    pk = synth.pack(problem, scs)
    solver = tadmm.Solver(tadmm.make_params(problem))
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag)
    prep.sqp(tadmm.MODE_BATCHED, max_rounds=max_rounds, rtol=rtol, sep_tol=sep_tol)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = prep.sqp(tadmm.MODE_BATCHED, max_rounds=max_rounds, rtol=rtol, sep_tol=sep_tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = st.cpu().numpy()
    status = prep.o["status"].cpu().numpy()
    rounds = st[:, 0].astype(int)
    prep1 = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag)
    prep1.run(tadmm.MODE_BATCHED)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prep1.run(tadmm.MODE_BATCHED)
    torch.cuda.synchronize()
    d1 = time.perf_counter() - t1
    s1 = prep1.o["status"].cpu().numpy()
    solver.close()
    return [dict(study="sqp", scenarios=S, max_rounds=max_rounds, rtol=rtol, sep_tol=sep_tol,
                 ms=round(1e3 * dt, 2), scenario_sqp_solves_per_s=round(S / dt, 1),
                 rounds_mean=round(float(rounds.mean()), 3),
                 rounds_hist={str(r): int((rounds == r).sum()) for r in range(1, max_rounds + 1)},
                 stopping_rule_met=round(float(st[:, 1].mean()), 4),
                 last_round_admm_converged=round(float((status == tadmm.SCEN_CONVERGED).mean()), 4),
                 min_separation_median=round(float(np.median(st[:, 3])), 4),
                 per_iteration_normals=dict(ms=round(1e3 * d1, 2),
                                            admm_converged=round(float((s1 == tadmm.SCEN_CONVERGED).mean()), 4)))]


def rho_study(S: int = 4096) -> List[Dict]:
    """The benchmark's batch with the penalty fixed (rho = 1) and adapted by
    residual balancing (mu = 10, tau = 2, every iteration), each without and
    with over-relaxation (alpha = 1.6), with momentum (fast ADMM with
    restart, eta = 0.999), with a velocity box, and with the shared dynamics
    given per agent (the one-lane-per-agent local QP instead of the per-axis
    split): converged fraction, mean iterations, refactored stages and time."""
    import torch

    import synth
    import paper_2602_15838_amd as tadmm
    problem, scs = synth.config2(S=S)
    pk = synth.pack(problem, scs)
    recs = []
    adapt = dict(adaptive_rho=True, rho_mu=10.0, rho_tau=2.0, rho_every=1)
    dyn = dict(agent_A=np.tile(problem.A.reshape(1, -1), (int(pk.n_agents.sum()), 1)),
               agent_B=np.tile(problem.B.reshape(1, -1), (int(pk.n_agents.sum()), 1)))
    for name, kw in (("fixed", {}), ("adaptive", adapt), ("fixed, alpha 1.6", dict(alpha=1.6)),
                     ("adaptive, alpha 1.6", dict(adapt, alpha=1.6)), ("momentum", dict(momentum=True)),
                     ("velocity box |v| <= 2", dict(state_box=True, s_lo=(-2.0, -2.0), s_hi=(2.0, 2.0))),
                     ("shared dynamics given per agent (one lane per agent)", dict(per_agent=True))):
        per_agent = kw.pop("per_agent", False)
        solver = tadmm.Solver(tadmm.make_params(problem, **kw))
        prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag,
                              **(dyn if per_agent else {}))
        prep.run(tadmm.MODE_BATCHED)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prep.run(tadmm.MODE_BATCHED)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = prep.o["status"].cpu().numpy()
        it = prep.o["iters"].cpu().numpy()
        cnt = prep.o["counters"].cpu().numpy()
        recs.append(dict(study="rho", penalty=name, scenarios=S, ms=round(1e3 * dt, 2),
                         scenario_solves_per_s=round(S / dt, 1),
                         converged=round(float((st == tadmm.SCEN_CONVERGED).mean()), 4),
                         mean_iters=round(float(it.mean()), 2),
                         mean_iters_converged=round(float(it[st == tadmm.SCEN_CONVERGED].mean()), 2),
                         refactored_axis_stages=int(cnt[:, 1].sum())))
        solver.close()
    return recs


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--ablation", action="store_true")
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--sqp", action="store_true")
    ap.add_argument("--rho", action="store_true")
    ap.add_argument("--seeds", type=int, default=20)
    args = ap.parse_args(argv)
    if not (args.ablation or args.sweep or args.sqp or args.rho):
        args.ablation = args.sweep = args.sqp = args.rho = True
    import torch
    torch.cuda.set_device(0)
    if args.ablation:
        for rec in ablation(args.seeds):
            print(json.dumps(rec), flush=True)
    if args.sweep:
        for rec in sweep():
            print(json.dumps(rec), flush=True)
    if args.sqp:
        for rec in sqp_study():
            print(json.dumps(rec), flush=True)
    if args.rho:
        for rec in rho_study():
            print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    sys.exit(main())
