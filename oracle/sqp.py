"""SQP outer loop around the FP64 ADMM: the separation constraints
re-linearized about each round's solution.

TEST INFRASTRUCTURE ONLY (see the package docstring): imported by the tests
alone; the product path never uses it.

Every separation constraint ||p_i,t - p_j,t|| >= d_min of Eq. 1 is replaced
by the half-plane n'(p_i,t - p_j,t) >= d_min with a frozen unit normal n, the
convexification of Sec. III-A.  Round 0 takes the normals of the reference
trajectories.  Every round solves that convex QP with the ADMM (normals
frozen), and the next round takes the normals of its solution.  The loop
stops the way the centralized solvers of the experiments do (Sec. V-A):
once the relative change of the objective of Eq. 1 between two rounds is
below rtol and the solution keeps every pair at least d_min apart at every
step (to sep_tol); otherwise after max_rounds.  Each round here starts cold
(from the references), as the oracle's ADMM always does.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np

import oracle


def objective(problem, x, u, xref, q_diag, r_diag) -> float:
    """Objective of Eq. 1 for one scenario: sum over agents of
    sum_{t<T} ||x_t - r_t||_Q^2 + ||u_t||_R^2, plus ||x_T - r_T||_{Q_T}^2 with
    Q_T = qT_scale Q.  x, xref [N][T+1][nx], u [N][T][nu]; q_diag, r_diag
    shared ([nx], [nu]) or per agent ([N][nx], [N][nu])."""
    x = np.asarray(x, np.float64)
    u = np.asarray(u, np.float64)
    e = x - np.asarray(xref, np.float64)
    N = x.shape[0]
    q = np.broadcast_to(np.asarray(q_diag, np.float64), (N, x.shape[2]))
    r = np.broadcast_to(np.asarray(r_diag, np.float64), (N, u.shape[2]))
    J = 0.0
    for i in range(N):
        T = u.shape[1]
        for t in range(T):
            J += float(e[i, t] @ (q[i] * e[i, t])) + float(u[i, t] @ (r[i] * u[i, t]))
        J += problem.qT_scale * float(e[i, T] @ (q[i] * e[i, T]))
    return J


def min_separation(x, dp: int) -> float:
    """Smallest distance between two agents' positions over the steps
    t = 1..T (the constrained steps); inf for a single agent."""
    x = np.asarray(x, np.float64)
    N = x.shape[0]
    best = np.inf
    for i in range(N):
        for j in range(i + 1, N):
            d = np.linalg.norm(x[i, 1:, :dp] - x[j, 1:, :dp], axis=1)
            best = min(best, float(d.min()))
    return best


def sqp_solve(problem, scenarios: Sequence, opts: Optional[oracle.OracleOptions] = None, max_rounds: int = 10,
              rtol: float = 1e-4, sep_tol: float = 1e-2, inputs=None, threads: int = 0) -> List[Dict[str, object]]:
    """The SQP loop on every scenario.  Per scenario: the last round's ADMM
    result (x, u, w, pair_active, status, iters), `rounds` (solves run),
    `converged` (the stopping rule met), the objective and the minimum
    separation of every round, and the normals of the last round."""
    base = opts or oracle.OracleOptions()
    o = oracle.OracleOptions(**{**base.__dict__, "normal_mode": oracle.NORMAL_FROZEN})
    S = len(scenarios)
    ins = [(sc.x0(), sc.xref()) if inputs is None else inputs[k] for k, sc in enumerate(scenarios)]
    qd = [sc.agent_q if getattr(sc, "agent_q", None) is not None else
          (problem.q_diag if sc.q_diag is None else sc.q_diag) for sc in scenarios]
    rd = [sc.agent_r if getattr(sc, "agent_r", None) is not None else
          (problem.r_diag if sc.r_diag is None else sc.r_diag) for sc in scenarios]
    out: List[Optional[Dict[str, object]]] = [None] * S
    hist = [dict(objective=[], min_sep=[]) for _ in range(S)]
    normals: List[Optional[np.ndarray]] = [None] * S      # round 0: the reference normals
    active = list(range(S))
    for rnd in range(max_rounds):
        if not active:
            break
        res = oracle.solve_batch(problem, [scenarios[k] for k in active], o, threads=threads,
                                 normals=None if rnd == 0 else [normals[k] for k in active],
                                 inputs=[ins[k] for k in active])
        still = []
        for k, r in zip(active, res):
            sc = scenarios[k]
            J = objective(problem, r["x"], r["u"], np.asarray(ins[k][1]).reshape(sc.N, sc.T + 1, -1), qd[k], rd[k])
            ms = min_separation(r["x"], problem.dp)
            h = hist[k]
            done = (len(h["objective"]) >= 1 and abs(J - h["objective"][-1]) <= rtol * max(abs(J), 1e-300)
                    and ms >= problem.d_min - sep_tol)
            h["objective"].append(J)
            h["min_sep"].append(ms)
            used = normals[k]
            out[k] = dict(r, rounds=rnd + 1, converged=done, objective=list(h["objective"]),
                          min_sep=list(h["min_sep"]), normals=used)
            if not done:
                normals[k] = oracle.relinearize(problem, sc, r["x"], inputs=ins[k])
                still.append(k)
        active = still
    return out  # type: ignore[return-value]
