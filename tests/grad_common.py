"""Equality-QP instances for the gradient tests, built from the oracle alone.

A case is a scenario whose oracle solve (normals re-linearized every
iteration) converged; its final positions fix the normals, the oracle then
solves the QP with those normals frozen to a tight tolerance, and the working
sets and binding half-planes of that solve define the equality QP.  A case is
kept only if the equality QP is certified to be the minimizer of the
frozen-normal QP (KKT conditions) and its KKT matrix is well conditioned (the
held constraints are independent, so the x0 gradient is unique)."""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

import oracle
from oracle import grad as G
from tests.gpu_common import Fp32Problem, fp32_inputs

CERT_TOL = 1e-7
COND_MAX = 1e10


def pair_index(N):
    return [(i, j) for i in range(N) for j in range(i + 1, N)]


def final_normals(x, xref, dp):
    """Unit normals (p_i - p_j)/|p_i - p_j| at the final positions, [P][T][dp]
    in canonical pair order (i < j lexicographic, t = 1..T).  Positions closer
    than 1e-6 take the normalized reference difference instead."""
    N, T1 = x.shape[0], x.shape[1]
    out = np.zeros((N * (N - 1) // 2, T1 - 1, dp))
    for p, (i, j) in enumerate(pair_index(N)):
        for t in range(1, T1):
            d = x[i, t, :dp] - x[j, t, :dp]
            nn = np.linalg.norm(d)
            if nn < 1e-6:
                d = xref[i, t, :dp] - xref[j, t, :dp]
                nn = np.linalg.norm(d)
            out[p, t - 1] = d / nn
    return out


def instance(problem, sc, res, normals, inputs=None) -> G.EqpInstance:
    """EqpInstance from a frozen-normal oracle result."""
    N, T = sc.N, sc.T
    x0, xref = (sc.x0(), sc.xref()) if inputs is None else inputs
    q = problem.q_diag if sc.q_diag is None else sc.q_diag
    r = problem.r_diag if sc.r_diag is None else sc.r_diag
    nd, active = {}, []
    for p, (i, j) in enumerate(pair_index(N)):
        for t in range(1, T + 1):
            nd[(i, j, t)] = np.asarray(normals[p, t - 1], dtype=np.float64)
            if res["pair_active"][p, t - 1]:
                active.append((i, j, t))
    return G.EqpInstance(A=np.asarray(problem.A, np.float64), B=np.asarray(problem.B, np.float64),
                         u_lo=np.asarray(problem.u_lo, np.float64), u_hi=np.asarray(problem.u_hi, np.float64),
                         qT_scale=float(problem.qT_scale), d_min=float(problem.d_min),
                         x0=np.asarray(x0, np.float64).copy(), xref=np.asarray(xref, np.float64).copy(),
                         logq=np.log(np.asarray(q, np.float64)), logr=np.log(np.asarray(r, np.float64)),
                         W=res["w"].astype(np.int64), active=active, normals=nd)


@dataclasses.dataclass
class Case:
    sid: int
    sc: object
    normals: np.ndarray          # [P][T][dp], the frozen normals
    res: dict                    # oracle result with the normals frozen
    ins: G.EqpInstance
    cert: tuple


def build_cases(problem, scenarios: Sequence, ids: Sequence[int], want: int, threads: int = 0,
                per_iter_max: int = 1000, frozen_eps: float = 1e-8, frozen_max: int = 3000,
                fp32: bool = True) -> List[Case]:
    """Up to `want` certified cases, in the order of `ids`.  With `fp32` the
    oracle solves the instance rounded to FP32 (what the device receives)."""
    P = Fp32Problem(problem) if fp32 else problem
    inputs = [fp32_inputs(sc) if fp32 else (sc.x0(), sc.xref()) for sc in scenarios]
    o1 = oracle.OracleOptions()
    o1.max_iter = per_iter_max
    r1 = oracle.solve_batch(P, scenarios, o1, threads=threads, inputs=inputs)
    keep = [k for k, r in enumerate(r1) if r["status"] == oracle.CONVERGED]
    nrm = [final_normals(r1[k]["x"], inputs[k][1], problem.dp) for k in keep]
    if fp32:   # the device receives the normals in FP32
        nrm = [n.astype(np.float32).astype(np.float64) for n in nrm]
    o2 = oracle.OracleOptions()
    o2.normal_mode = oracle.NORMAL_FROZEN
    o2.eps_abs = o2.eps_rel = frozen_eps
    o2.max_iter = frozen_max
    r2 = oracle.solve_batch(P, [scenarios[k] for k in keep], o2, threads=threads, normals=nrm,
                            inputs=[inputs[k] for k in keep])
    cases = []
    for n_k, k in enumerate(keep):
        res = r2[n_k]
        if res["status"] != oracle.CONVERGED:
            continue
        ins = instance(P, scenarios[k], res, nrm[n_k], inputs[k])
        if not ins.active:
            continue
        if G.kkt_condition(ins) > COND_MAX:
            continue
        cert = G.kkt_certificate(ins)
        if max(cert) > CERT_TOL:
            continue
        cases.append(Case(ids[k], scenarios[k], nrm[n_k], res, ins, cert))
        if len(cases) >= want:
            break
    return cases


def tracking_loss_grads(ins: G.EqpInstance, x, u, pref):
    """L = sum_{i,k} ||p_i,k - pref_i,k||^2 (k = 0..T) and its partials."""
    dp = ins.nu
    gx = np.zeros_like(x)
    gx[:, :, :dp] = 2.0 * (x[:, :, :dp] - pref)
    return float(np.sum((x[:, :, :dp] - pref) ** 2)), gx, np.zeros_like(u)


def rel_err(a, b) -> float:
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
