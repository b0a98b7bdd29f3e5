"""Convergence of the FP64 oracle's ADMM on the named workloads.

TEST INFRASTRUCTURE ONLY (see the package docstring): a study of the
oracle, run by hand (``python -m oracle.convergence_study``); the product
path never uses it.

For each workload it reports, with the stopping rule of Sec. V-A
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


def study(name, p, scs, max_iter, K, threads=0, sqp_rounds=10):
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


def main(argv):
    which = argv[1:] or ["0", "1", "2", "4"]
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
        study("config4", p, s, 60, 40, sqp_rounds=0)


if __name__ == "__main__":
    main(sys.argv)
