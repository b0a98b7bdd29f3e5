#!/usr/bin/env python3
"""Throughput of the ADMM hot path on one MI355X.

Workload: 4096 independent scenarios (agents N ~ U{2..32}, horizon
T ~ U{10..40}, 2-D double integrator, random starts/goals in [-5,5]^2 with
1.0 separation), solved to the 1e-4 residual test (at most 200 iterations).
A step = one batched solve of the whole batch (persistent kernel launched
through a cached hipGraph), inputs already resident in HBM.

Prints one JSON line: scenario solves/s (value), agent-QP solves/s, the plain
per-scenario path on a sample, the roofline of the persistent kernel and the
FP64 oracle timed on the host cores on a bounded sample.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per unit, the method's own count for the joint per-agent
# local QP: per agent-stage and active-set pass (affine backward sweep with
# the cached factors, rollout, ratio test) 190 flops in 2-D (380 in 3-D) and
# 152 B (324 B) when the stage factors and affine terms stream from HBM; per
# refactored agent-stage 520 (1400) flops and the same bytes; per pair-step
# (projection, dual update, residual pieces) 40 (55) flops and 8 B (the
# collapsed dual read and written).  With double-integrator dynamics the
# kernel solves each local QP as one problem per coordinate axis and its
# counters count axis-stages (dp per agent-stage), so the agent-stage
# figures are divided by dp.
_AGENT_STAGE = {2: dict(affine=(190.0, 152.0), refactor=(520.0, 152.0)),
                3: dict(affine=(380.0, 324.0), refactor=(1400.0, 324.0))}
FLOPS_PER_UNIT = {dp: dict(affine=_AGENT_STAGE[dp]["affine"][0] / dp, refactor=_AGENT_STAGE[dp]["refactor"][0] / dp,
                           pair=40.0 if dp == 2 else 55.0) for dp in (2, 3)}
BYTES_PER_UNIT = {dp: dict(affine=_AGENT_STAGE[dp]["affine"][1] / dp, refactor=_AGENT_STAGE[dp]["refactor"][1] / dp,
                           pair=8.0) for dp in (2, 3)}
PEAK_HBM_GBS = 8000.0             # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector (packed) peak
PEAK_FP32_UNPACKED_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
METRIC = "ADMM scenario solves/s + agent-QP solves/s at 1e-4 residual, batched vs plain"
# HBM traffic of one persistent-kernel launch, from rocprofv3 counter runs
# (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size); valid
# only for the kernel sources it was measured on
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_admm_persistent_config2_hbm_traffic.txt")
COPY_BYTES = 256 << 20


def source_digest() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2602_15838_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(scenarios: int):
    """Bytes per launch from the committed counter summary, or None when it is
    missing, for another batch size, or older than the kernel sources."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    kv = {}
    for line in open(PMC_SUMMARY):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv.get("source_sha256") != source_digest() or int(kv.get("scenarios", -1)) != scenarios:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def step_stats(v):
    v = np.asarray(v, dtype=np.float64)
    return {"median": round(float(np.median(v)), 4), "std": round(float(v.std()), 4),
            "min": round(float(v.min()), 4), "max": round(float(v.max()), 4)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--scenarios", type=int, default=4096)
    ap.add_argument("--plain-sample", type=int, default=-1, help="scenarios of the plain path (-1: the whole batch)")
    ap.add_argument("--cpu-sample", type=int, default=640)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="skip the workgroup-size autotuner of the setup")
    ap.add_argument("--block-threads", type=int, default=0)
    ap.add_argument("--cpu-variant-sample", type=int, default=24)
    ap.add_argument("--profile-steps", action="store_true", help="print one line per step (for profiler runs)")
    ap.add_argument("--no-scale", action="store_true", help="skip the 3-D single-scenario (128 agents) line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 256 MiB (the reference for HBM counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (the multi-GPU sharding is a design, not a run)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_2602_15838_amd as tadmm
    import synth

    torch.cuda.set_device(0)
    t0 = time.time()
    problem, scs = synth.config2(S=args.scenarios)
    pk = synth.pack(problem, scs)
    Ns, Ts = pk.n_agents.astype(np.int64), pk.horizon.astype(np.int64)
    print(f"# generated {len(scs)} scenarios in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    solver = tadmm.Solver(tadmm.make_params(problem, block_threads=args.block_threads))
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag)
    tuned = None
    if not args.no_autotune and not args.block_threads:
        # untimed setup: time the candidate workgroup sizes on this batch and
        # keep the fastest in the context
        tuned = prep.autotune()
        print(f"# autotuned workgroup size {tuned}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        prep.run(tadmm.MODE_BATCHED)
    torch.cuda.synchronize()
    kms, wms = [], []
    t_start = time.perf_counter()
    for k in range(args.steps):
        t1 = time.perf_counter()
        kms.append(prep.run(tadmm.MODE_BATCHED))   # returns after the stream has synchronized
        wms.append(1e3 * (time.perf_counter() - t1))
        if args.profile_steps:
            print(f"# step {k} kernel {kms[-1]:.3f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_step = 1e3 * wall / args.steps
    res = prep.result()
    status = res["status"].cpu().numpy()
    iters = res["iters"].cpu().numpy().astype(np.int64)
    cnt = res["counters"].cpu().numpy().astype(np.float64)
    S = len(scs)
    scen_per_s = S / (ms_step / 1e3)
    conv_per_s = float((status == 0).sum()) / (ms_step / 1e3)
    agent_qp = float((Ns * iters).sum())
    agent_qp_per_s = agent_qp / (ms_step / 1e3)

    # roofline of the persistent kernel (HIP events around its graph launch on
    # the context's stream).  Below 1 algorithmic flop/B it sits far below the
    # FP32 ridge (157.3 TF / 8 TB/s = 19.7 flop/B): HBM is the bound.
    kernel_ms = float(np.mean(kms))
    fu, bu = FLOPS_PER_UNIT[problem.dp], BYTES_PER_UNIT[problem.dp]
    units = dict(affine=float(cnt[:, 2].sum()), refactor=float(cnt[:, 1].sum()), pair=float(cnt[:, 3].sum()))
    flops = sum(fu[k] * units[k] for k in units)
    nbytes = sum(bu[k] * units[k] for k in units)
    gbs = nbytes / (kernel_ms / 1e3) / 1e9
    tflops = flops / (kernel_ms / 1e3) / 1e12
    roofline = {"bound": "hbm", "achieved": round(gbs, 2), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 5), "traffic": measured_traffic(S),
                "kernel": "k_admm_persistent<4,2>", "kernel_ms": round(kernel_ms, 4),
                "algorithmic_bytes_per_launch": round(nbytes), "algorithmic_gflop_per_launch": round(flops / 1e9, 4),
                "alu": {"achieved": round(tflops, 4), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(tflops / PEAK_FP32_TFLOPS, 6),
                        "frac_of_unpacked_fp32": round(tflops / PEAK_FP32_UNPACKED_TFLOPS, 6)},
                "units_per_launch": {k: int(v) for k, v in units.items()}}

    out = {"metric": METRIC, "value": round(scen_per_s, 2),
           "unit": "scenario solves/s", "n_gpus": 1,
           # value counts every scenario run to termination: converged at 1e-4
           # or stopped by the 200-iteration cap (status_counts); the converged
           # ones alone, per second:
           "converged_scenario_solves_per_s": round(conv_per_s, 2), "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"ragged batch of {S} scenarios, N~U{{2..32}}, T~U{{10..40}}, 2-D double "
                                  f"integrator, rho=1, d_min=0.5, eps_abs=eps_rel=1e-4, max_iter=200",
                      "scenarios": S, "agents": int(Ns.sum()), "agent_stages": int((Ns * Ts).sum()),
                      "pair_steps": int((Ns * (Ns - 1) // 2 * Ts).sum()), "mode": "batched persistent + hipGraph",
                      "workgroup_threads": int(tuned or args.block_threads or 128)},
           "agent_qp_solves_per_s": round(agent_qp_per_s, 1),
           "converged_fraction": round(float((status == 0).mean()), 4),
           "status_counts": {str(k): int((status == k).sum()) for k in range(4)},
           "mean_iters": round(float(iters.mean()), 2),
           "step_ms": step_stats(wms), "kernel_ms": step_stats(kms),
           # passes of the per-axis problems, per axis problem solved
           "active_set_passes_per_axis_qp": round(float(cnt[:, 0].sum()) / max(agent_qp * problem.dp, 1.0), 4),
           "phase_time_split": {k: round(float(cnt[:, c].sum()) / max(float(cnt[:, 4:7].sum()), 1.0), 4)
                                for k, c in (("x_update", 4), ("pair", 5), ("test", 6))},
           # mean over scenarios of the time one workgroup spends per ADMM iteration in each phase
           "phase_us_per_iteration": {k: round(float(np.mean(cnt[:, c] / np.maximum(iters, 1))) / 100.0, 3)
                                      for k, c in (("x_update", 4), ("pair", 5), ("test", 6))},
           "roofline": roofline}

    if not args.no_plain and args.plain_sample != 0:
        n_plain = S if args.plain_sample < 0 else min(args.plain_sample, S)
        ids = list(range(n_plain))
        sub = [scs[i] for i in ids]
        ps = synth.pack(problem, sub)
        # warm-up on the first scenarios, then one timed pass over the sample
        w = synth.pack(problem, sub[:4])
        solver.prepare(w.n_agents, w.horizon, w.x0, w.xref, w.q_diag, w.r_diag).run(tadmm.MODE_PLAIN)
        pprep = solver.prepare(ps.n_agents, ps.horizon, ps.x0, ps.xref, ps.q_diag, ps.r_diag)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        pprep.run(tadmm.MODE_PLAIN)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - tp
        pit = pprep.o["iters"].cpu().numpy().astype(np.int64)
        if n_plain == S:
            dtb = ms_step / 1e3
        else:
            bprep = solver.prepare(ps.n_agents, ps.horizon, ps.x0, ps.xref, ps.q_diag, ps.r_diag)
            bprep.run(tadmm.MODE_BATCHED)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            bprep.run(tadmm.MODE_BATCHED)
            torch.cuda.synchronize()
            dtb = time.perf_counter() - tb
        out["plain"] = {"sample": f"scenarios 0..{len(ids) - 1} of the batch, solved one by one (host loop, "
                                  f"3 launches + 1 sync per iteration), one timed pass",
                        "scenario_solves_per_s": round(len(ids) / dtp, 2),
                        "agent_qp_solves_per_s": round(float((ps.n_agents * pit).sum()) / dtp, 1),
                        "batched_same_scenarios_scenario_solves_per_s": round(len(ids) / dtb, 2),
                        "batched_over_plain_same_scenarios": round(dtp / dtb, 1)}
        print(f"# plain path {len(ids)} scenarios in {dtp:.2f}s", file=sys.stderr, flush=True)

    if not args.no_cpu and args.cpu_sample > 0:
        import oracle
        ids = list(range(min(args.cpu_sample, S)))
        sub = [scs[i] for i in ids]
        th = oracle.max_threads()
        tc = time.perf_counter()
        ro = oracle.solve_batch(problem, sub, threads=th)
        dtc = time.perf_counter() - tc
        oit = np.array([r["iters"] for r in ro], dtype=np.int64)
        # the converged fraction at 1e-4 on this sample, beside the device's
        # on the same scenarios (the oracle solves the FP64 instance)
        ost = np.array([r["status"] for r in ro])
        out["converged_fraction_sample"] = {"scenarios": len(ids),
                                            "device": round(float((status[ids] == 0).mean()), 4),
                                            "oracle": round(float((ost == oracle.CONVERGED).mean()), 4)}
        out["cpu_baseline"] = {"value": round(len(ids) / dtc, 3), "unit": "scenario solves/s", "cores": int(th),
                               "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
                               "sample": f"scenarios 0..{len(ids) - 1} of the batch, FP64 dense-KKT oracle, OpenMP "
                                         f"over scenarios, {dtc:.1f}s",
                               "agent_qp_solves_per_s": round(float((np.array([s.N for s in sub]) * oit).sum()) / dtc, 1)}
        print(f"# cpu oracle sample {len(ids)} scenarios in {dtc:.1f}s on {th} threads", file=sys.stderr, flush=True)
        # the oracle on one core, and without its factor reuse (the CPU
        # mirror of the hotstart), on a smaller sample of the same batch
        vids = ids[:min(len(ids), args.cpu_variant_sample)]
        vsub = [scs[i] for i in vids]
        var = {"sample": f"scenarios 0..{len(vids) - 1} of the batch", "unit": "scenario solves/s"}
        for name, thr, opts in (("threads_all_lu_reuse", th, oracle.OracleOptions()),
                                ("threads_1_lu_reuse", 1, oracle.OracleOptions()),
                                ("threads_all_no_lu_reuse", th, oracle.OracleOptions(lu_reuse=False))):
            tv = time.perf_counter()
            oracle.solve_batch(problem, vsub, opts, threads=thr)
            var[name] = round(len(vids) / (time.perf_counter() - tv), 3)
        var["threads_all"] = int(th)
        out["cpu_oracle_variants"] = var
        print(f"# cpu oracle variants on {len(vids)} scenarios: {var}", file=sys.stderr, flush=True)

    if not args.no_scale:
        # the 3-D scale workload: one scenario of 128 agents, T = 50 (8128 pairs
        # x 50 steps), through the many-workgroup mode and, for comparison,
        # the persistent kernel (one workgroup) and the plain host loop
        p4, sc4 = synth.config4()
        k4 = synth.pack(p4, sc4)
        s4 = tadmm.Solver(tadmm.make_params(p4))
        pr4 = s4.prepare(k4.n_agents, k4.horizon, k4.x0, k4.xref, k4.q_diag, k4.r_diag)
        scale = {"workload": "1 scenario, 128 agents on a radius-12 Fibonacci sphere to antipodes, 3-D double "
                             "integrator, T=50, |u|<=3, max_iter=200"}
        for name, mode in (("wide", tadmm.MODE_WIDE), ("persistent", tadmm.MODE_BATCHED), ("plain", tadmm.MODE_PLAIN)):
            pr4.run(mode)
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            pr4.run(mode)
            torch.cuda.synchronize()
            scale[f"{name}_ms_per_solve"] = round(1e3 * (time.perf_counter() - t4), 2)
        it4 = int(pr4.o["iters"][0])
        scale["iterations"] = it4
        # the derivative of the same solve: polish on the frozen active sets,
        # then the adjoint of a seeded loss gradient
        gx = torch.as_tensor(np.random.default_rng(4).standard_normal(tuple(pr4.o["x"].shape)),
                             dtype=torch.float32, device=pr4.o["x"].device)
        pr4.polish()                      # warm-up (a solve is polished once)
        pr4.run(tadmm.MODE_WIDE)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        pr4.polish()
        torch.cuda.synchronize()
        scale["polish_ms"] = round(1e3 * (time.perf_counter() - t4), 2)
        pr4.adjoint(gx)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        pr4.adjoint(gx)
        torch.cuda.synchronize()
        scale["adjoint_ms"] = round(1e3 * (time.perf_counter() - t4), 2)
        scale["agent_qp_solves_per_s_wide"] = round(128 * it4 / (scale["wide_ms_per_solve"] / 1e3), 1)
        out["scale_workload"] = scale
        s4.close()
        print(f"# 3-D scale workload: {scale}", file=sys.stderr, flush=True)

    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 4, device="cuda")
        dst = torch.empty_like(src)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        dst.copy_(src)
        torch.cuda.synchronize()
        ev0.record()
        dst.copy_(src)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        out["copy_calibration"] = {"bytes_read": COPY_BYTES, "bytes_written": COPY_BYTES, "ms": round(ms, 4),
                                   "GB_per_s": round(2 * COPY_BYTES / (ms / 1e3) / 1e9, 1), "dispatches": 2}
        print(f"# copy calibration {COPY_BYTES} B in {ms:.3f} ms", file=sys.stderr, flush=True)

    print(json.dumps(out))
    solver.close()


if __name__ == "__main__":
    main()
