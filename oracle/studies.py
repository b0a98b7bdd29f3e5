"""Studies of the FP64 oracle's ADMM, run by hand:

    python -m oracle.studies convergence [0 1 2 4]
    python -m oracle.studies ablation

TEST INFRASTRUCTURE ONLY (see the package docstring); the product path never
uses it.

convergence: for each named workload it reports, with the stopping rule of Sec. V-A
(eps_abs = eps_rel = 1e-4):
  * the residual norms ||r||, ||s|| and their tolerances at checkpoints of a
    run with normals of the iterates (the default reading), and the
    iteration at which the test passed, if it did within the cap;
  * between two consecutive iterates x^K and x^(K+1), how many pair-steps
    turned their normal (the linearization of ||p_i - p_j|| >= d_min about
    the iterate) by more than 10 and 90 degrees, and how many of those
    half-planes were violated (active) at step K;
  * the same ADMM with the normals frozen at those of x^K (a convex QP):
    whether and when it passes the same test;
  * the SQP loop of oracle/sqp.py (rounds of frozen-normal solves).
Prints one JSON object per workload.

ablation (Sec. V-B, Table II): the oracle's active-set passes and LU
factorizations per solve for the three start strategies of the paper's
comparison, on the crossings of the device's ablation study (the same seeded
scenarios, 2-14 agents, T = 20): Base (every local QP from u = 0 and an empty
working set, no factor reuse), Hotstart (iterations >= 2 from the previous
iterate and working set, LU reuse while the working set is unchanged) and
Turbo (Hotstart plus the clipped unconstrained solution as the start of
iteration 1).  Prints one JSON object per agent count and variant.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

import oracle
import synth
from oracle import sqp

CHECK = (1, 10, 50, 100, 200, 500, 1000, 2000)


def _angles(n0, n1):
    c = np.clip(np.sum(n0 * n1, axis=-1), -1.0, 1.0)
    return np.degrees(np.arccos(c))


def feasibility_margin(p, sc, normals):
    """Largest m such that every half-plane n'(p_i,t - p_j,t) >= d_min + m
    (t = 1..T, the given normals [P][T][dp]) holds for some inputs in the
    box, the positions being those of the dynamics from the scenario's
    starts (a linear program, HiGHS).  m < 0: the frozen half-planes admit
    no trajectory at all, so no ADMM iterate can satisfy them."""
    import scipy.optimize
    import scipy.sparse
    N, T, nx, nu, dp = sc.N, sc.T, p.nx, p.nu, p.dp
    A, B = np.asarray(p.A), np.asarray(p.B)
    C = np.eye(nx)[:dp]
    pw = [np.eye(nx)]
    for _ in range(T):
        pw.append(A @ pw[-1])
    G = [C @ pw[k] @ B for k in range(T)]             # position response k steps after an input
    x0 = np.asarray(sc.x0(), np.float64).reshape(N, nx)
    nv = N * T * nu
    rows, cols, vals, rhs = [], [], [], []
    r = 0
    pidx = 0
    for i in range(N):
        for j in range(i + 1, N):
            for t in range(1, T + 1):
                n = normals[pidx, t - 1]
                for s_ in range(t):
                    g = n @ G[t - 1 - s_]
                    for a in range(nu):
                        if g[a] != 0.0:
                            rows += [r, r]
                            cols += [(i * T + s_) * nu + a, (j * T + s_) * nu + a]
                            vals += [-g[a], g[a]]
                rows.append(r)
                cols.append(nv)
                vals.append(1.0)
                rhs.append(float(n @ (C @ pw[t] @ (x0[i] - x0[j]))) - p.d_min)
                r += 1
            pidx += 1
    Aub = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(r, nv + 1))
    c = np.zeros(nv + 1)
    c[-1] = -1.0
    bounds = [(float(p.u_lo[a]), float(p.u_hi[a])) for _ in range(N * T) for a in range(nu)] + [(None, 10.0)]
    res = scipy.optimize.linprog(c, A_ub=Aub, b_ub=np.asarray(rhs), bounds=bounds, method="highs")
    return float(res.x[-1]) if res.status == 0 else float("nan")


def study(name, p, scs, max_iter, K, threads=0, sqp_rounds=10, lp=True):
    t0 = time.time()
    opts = oracle.OracleOptions(max_iter=max_iter)
    runs = oracle.solve_batch(p, scs, opts, threads=threads)
    rep = dict(workload=name, scenarios=len(scs), max_iter=max_iter)
    conv = [r["iters"] for r in runs if r["status"] == oracle.CONVERGED]
    rep["converged"] = len(conv)
    rep["converged_iters"] = sorted(conv)[:20]
    if len(scs) == 1:
        h = runs[0]["hist"]
        rep["history"] = {k: [float(v) for v in h[k - 1]] for k in CHECK if k <= len(h)}
    else:
        for cap in (200, 500, 1000, max_iter):
            rep[f"converged_within_{cap}"] = sum(1 for r in runs if r["status"] == oracle.CONVERGED and r["iters"] <= cap)
    # normals of two consecutive iterates, and the frozen-normal QP at x^K
    flips = dict(pair_steps=0, over_10deg=0, over_90deg=0, active=0, active_over_10deg=0, active_over_90deg=0)
    frozen_conv, frozen_iters = 0, []
    for sc in scs:
        a = oracle.solve(p, sc, oracle.OracleOptions(fixed_iters=K), keep_zl=False, threads=max(threads, 1))
        b = oracle.solve(p, sc, oracle.OracleOptions(fixed_iters=K + 1), keep_zl=False, threads=max(threads, 1))
        if sc.N < 2:
            continue
        n0 = oracle.relinearize(p, sc, a["x"])
        n1 = oracle.relinearize(p, sc, b["x"])
        ang = _angles(n0, n1)
        act = a["pair_active"].astype(bool)
        flips["pair_steps"] += int(ang.size)
        flips["over_10deg"] += int((ang > 10).sum())
        flips["over_90deg"] += int((ang > 90).sum())
        flips["active"] += int(act.sum())
        flips["active_over_10deg"] += int((ang[act] > 10).sum())
        flips["active_over_90deg"] += int((ang[act] > 90).sum())
        f = oracle.solve(p, sc, oracle.OracleOptions(normal_mode=oracle.NORMAL_FROZEN, max_iter=max_iter),
                         normals=n0, threads=max(threads, 1))
        if f["status"] == oracle.CONVERGED:
            frozen_conv += 1
            frozen_iters.append(f["iters"])
    rep[f"normal_turns_between_iterates_{K}_and_{K + 1}"] = flips
    if lp:
        # feasibility of the frozen half-planes of the references and of x^K
        # for the scenarios that did not converge within the cap
        marg = []
        for sc, r in zip(scs, runs):
            if sc.N < 2 or r["status"] == oracle.CONVERGED:
                continue
            a = oracle.solve(p, sc, oracle.OracleOptions(fixed_iters=K), threads=max(threads, 1))
            marg.append((feasibility_margin(p, sc, oracle.relinearize(p, sc, sc.xref())),
                         feasibility_margin(p, sc, oracle.relinearize(p, sc, a["x"]))))
        rep["unconverged_feasibility_margin"] = dict(
            scenarios=len(marg), reference_normals=[round(m[0], 4) for m in marg][:20],
            iterate_normals=[round(m[1], 4) for m in marg][:20],
            infeasible_at_iterate=sum(1 for m in marg if m[1] < 0))
    rep[f"frozen_at_iterate_{K}"] = dict(converged=frozen_conv, iters=sorted(frozen_iters)[:20])
    if sqp_rounds:
        res = sqp.sqp_solve(p, scs, oracle.OracleOptions(max_iter=max_iter), max_rounds=sqp_rounds, threads=threads)
        rep["sqp"] = dict(stopping_rule_met=sum(1 for r in res if r["converged"]),
                          rounds=[r["rounds"] for r in res][:20],
                          last_round_admm_converged=sum(1 for r in res if r["status"] == oracle.CONVERGED),
                          min_separation=[round(r["min_sep"][-1], 4) for r in res][:20])
    rep["seconds"] = round(time.time() - t0, 1)
    print(json.dumps(rep), flush=True)
    return rep


ABLATION = {"base": dict(warm_start=False, hotstart=False, lu_reuse=False),
            "hotstart": dict(warm_start=False, hotstart=True, lu_reuse=True),
            "turbo": dict(warm_start=True, hotstart=True, lu_reuse=True)}


def ablation_scenarios(N, seeds, config_id=5):
    """The device study's crossings: N agents, T = 20, random box starts and
    goals, seeds 1000 N + s of its seed stream."""
    p = synth.ProblemParams(dp=2, u_max=2.0)
    return p, [synth.random_box(synth.rng_for(config_id, 1000 * N + s), N, 20) for s in range(seeds)]


def ablation(agents=(2, 4, 6, 10, 14), seeds=20, threads=0):
    out = []
    for N in agents:
        p, scs = ablation_scenarios(N, seeds)
        for name, flags in ABLATION.items():
            t0 = time.time()
            res = oracle.solve_batch(p, scs, oracle.OracleOptions(**flags), threads=threads)
            rec = dict(study="oracle_ablation", agents=N, variant=name, seeds=seeds,
                       admm_iters=round(float(np.mean([r["iters"] for r in res])), 2),
                       converged=round(float(np.mean([r["status"] == oracle.CONVERGED for r in res])), 3),
                       active_set_passes=round(float(np.mean([r["as_passes"] for r in res])), 1),
                       lu_factorizations=round(float(np.mean([r["lu_factorizations"] for r in res])), 1),
                       seconds=round(time.time() - t0, 2))
            print(json.dumps(rec), flush=True)
            out.append(rec)
    return out


def main(argv):
    if len(argv) > 1 and argv[1] == "ablation":
        ablation()
        return
    which = [a for a in argv[1:] if a != "convergence"] or ["0", "1", "2", "4"]
    if "0" in which:
        p, s = synth.config0()
        study("config0", p, s, 2000, 200)
    if "1" in which:
        p, s = synth.config1()
        study("config1", p, s, 2000, 200)
    if "2" in which:
        p, s = synth.config2(S=64)
        study("config2 sample (scenarios 0..63)", p, s, 1000, 200, sqp_rounds=5)
    if "4" in which:
        p, s = synth.config4()
        study("config4", p, s, 60, 40, sqp_rounds=0, lp=False)


if __name__ == "__main__":
    main(sys.argv)
