"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare it with the FP64 oracle."""
from __future__ import annotations

import numpy as np

import oracle
import synth

# Parity bar: relative trajectory error over (x, u) of a scenario (FP32 path
# against the FP64 oracle).
REL_TOL = 1e-4
# A working-set entry or a half-plane counts as marginal (excluded from the
# identity check) when its multiplier and its slack are both this small.
MARGIN = 1e-5


def gpu_solve(problem, scs, mode=None, normals=None, solver_kw=None, return_prep=False, history=False):
    import paper_2602_15838_amd as tadmm
    mode = tadmm.MODE_BATCHED if mode is None else mode
    pk = synth.pack(problem, scs)
    solver = tadmm.Solver(tadmm.make_params(problem, **(solver_kw or {})))
    nrm = None if normals is None else np.concatenate([np.asarray(n).reshape(-1, problem.nu) for n in normals])
    prep = solver.prepare(pk.n_agents, pk.horizon, pk.x0, pk.xref, pk.q_diag, pk.r_diag, nrm, agent_q=pk.agent_q,
                          agent_r=pk.agent_r, agent_lo=pk.agent_lo, agent_hi=pk.agent_hi, agent_A=pk.agent_A,
                          agent_B=pk.agent_B, history=history)
    prep.run(mode)
    res = tadmm.split_outputs(prep.result(), pk.n_agents, pk.horizon, problem.nx, problem.nu)
    if return_prep:
        return res, prep, solver
    solver.close()
    return res


class Fp32Problem:
    """The problem constants exactly as the FP32 device path receives them
    (every value rounded to FP32), for the oracle to solve the same instance."""

    def __init__(self, p):
        r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
        f = lambda v: float(np.float32(v))
        self.dp, self.nx, self.nu, self.max_iter = p.dp, p.nx, p.nu, p.max_iter
        self.A, self.B = r(p.A), r(p.B)
        self.u_lo, self.u_hi, self.u_max = r(p.u_lo), r(p.u_hi), f(p.u_max)
        self.q_diag, self.r_diag = r(p.q_diag), r(p.r_diag)
        self.qT_scale, self.d_min, self.rho = f(p.qT_scale), f(p.d_min), f(p.rho)
        self.eps_abs, self.eps_rel = f(p.eps_abs), f(p.eps_rel)


def fp32_inputs(sc):
    """(x0, xref) of a scenario rounded to FP32, as the device receives them."""
    r = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    return r(sc.x0()), r(sc.xref())


def oracle_same_instance(problem, scs, opts, threads=0, keep_zl=False, normals=None):
    """Oracle on exactly the FP32 instance the device solves."""
    P32 = Fp32Problem(problem)
    if len(scs) == 1:
        return [oracle.solve(P32, scs[0], opts, normals=None if normals is None else normals[0],
                             threads=max(threads, 1), keep_zl=keep_zl, inputs=fp32_inputs(scs[0]))]
    return oracle.solve_batch(P32, scs, opts, threads=threads, normals=normals,
                              inputs=[fp32_inputs(sc) for sc in scs], keep_zl=keep_zl)


def self_sensitivity(problem, sc, opts, rel=1e-7, seed=0, threads=1) -> float:
    """The oracle's own response to a relative perturbation `rel` (below FP32
    rounding) of the start positions: how reproducible the result of this run
    is at all, whatever the arithmetic."""
    P32 = Fp32Problem(problem)
    x0, xref = fp32_inputs(sc)
    rng = np.random.default_rng(seed)
    x0p = x0.copy()
    x0p[:, :problem.dp] *= 1.0 + rel * rng.standard_normal(x0p[:, :problem.dp].shape)
    a = oracle.solve(P32, sc, opts, threads=threads, inputs=(x0, xref))
    b = oracle.solve(P32, sc, opts, threads=threads, inputs=(x0p, xref))
    return rel_traj_err(dict(x=b["x"], u=b["u"]), a)


def oracle_opts(solver_kw=None, lockstep=None):
    kw = dict(solver_kw or {})
    o = oracle.OracleOptions()
    for k in ("normal_mode", "mu_tol", "max_as_iter", "max_iter", "eps_abs", "eps_rel", "rho", "adaptive_rho",
              "rho_mu", "rho_tau", "rho_every", "state_box"):
        if k in kw:
            setattr(o, k, kw[k])
    if "riccati_warmstart" in kw:
        o.warm_start = bool(kw["riccati_warmstart"])
    if "hotstart" in kw:
        o.hotstart = bool(kw["hotstart"])
    if "alpha" in kw:
        o.alpha = float(np.float32(kw["alpha"]))
    if kw.get("momentum"):
        o.momentum = True
        o.mom_eta = float(np.float32(kw.get("mom_eta", 0.999)))
    for k in ("s_lo", "s_hi", "p_lo", "p_hi"):
        if k in kw:
            setattr(o, k, tuple(float(np.float32(v)) for v in kw[k]) + (0.0,) * (3 - len(kw[k])))
    if lockstep:
        o.fixed_iters = lockstep
    return o


def rel_traj_err(g, o) -> float:
    X = np.concatenate([o["x"].ravel(), o["u"].ravel()])
    Y = np.concatenate([g["x"].ravel(), g["u"].ravel()]).astype(np.float64)
    return float(np.linalg.norm(X - Y) / max(np.linalg.norm(X), 1e-30))


def working_set_marginal(problem, o) -> np.ndarray:
    """Bounds whose multiplier is tiny (degenerate) or whose input sits within
    MARGIN of the bound without being fixed there."""
    u, w, mu = o["u"], o["w"], o["mu"]
    scale = 1.0 + np.abs(mu).max()
    near = (np.abs(u - problem.u_lo) < MARGIN * problem.u_max) | (np.abs(u - problem.u_hi) < MARGIN * problem.u_max)
    return ((w != 0) & (np.abs(mu) < MARGIN * scale)) | ((w == 0) & near)


def pair_marginal(problem, sc, o, rho, normals=None) -> np.ndarray:
    """Half-planes whose violation v at the last consensus step is tiny:
    active: v = 2|lambda_ij|/rho; inactive: v = d_min - n'(z_ij - z_ji), with
    n the frozen normals [P][T][dp] when given, else those of the final
    positions."""
    N, T = sc.N, sc.T
    x, z, lam = o["x"], o["z"], o["lam"]
    out = np.zeros((N * (N - 1) // 2, T), dtype=bool)
    p = 0
    for i in range(N):
        for j in range(i + 1, N):
            if normals is not None:
                n = normals[p]
            else:
                d = x[i, 1:, :problem.dp] - x[j, 1:, :problem.dp]
                n = d / np.maximum(np.linalg.norm(d, axis=1, keepdims=True), 1e-300)
            act = o["pair_active"][p].astype(bool)
            v_act = 2.0 * np.linalg.norm(lam[i, j], axis=1) / rho
            v_in = problem.d_min - np.sum(n * (z[i, j] - z[j, i]), axis=1)
            v = np.where(act, v_act, v_in)
            out[p] = np.abs(v) < MARGIN * max(1.0, problem.d_min)
            p += 1
    return out


def compare(problem, sc, g, o, rho=None, check_sets=True, tol=REL_TOL, normals=None):
    """Assert parity of one scenario; returns a small report dict."""
    rho = problem.rho if rho is None else rho
    rel = rel_traj_err(g, o)
    rep = dict(rel=rel, iters=(g["iters"], o["iters"]), status=(g["status"], o["status"]))
    assert np.all(g["u"] >= problem.u_lo) and np.all(g["u"] <= problem.u_hi), "input outside the box"
    assert g["status"] != 2 or o["status"] == 2, f"active-set cap on the GPU only ({rep})"
    assert rel <= tol, f"N={sc.N} T={sc.T}: rel trajectory error {rel:.3e} > {tol:.0e} ({rep})"
    if check_sets:
        wm = working_set_marginal(problem, o)
        diff = (g["w"] != o["w"]) & ~wm
        assert not diff.any(), f"N={sc.N} T={sc.T}: working sets differ at {np.argwhere(diff)[:5].tolist()}"
        rep["w_marginal"] = int(wm.sum())
        if "z" in o and sc.N > 1:
            pm = pair_marginal(problem, sc, o, rho, normals)
            pdiff = (g["pair_active"] != o["pair_active"]) & ~pm
            assert not pdiff.any(), f"N={sc.N} T={sc.T}: active half-planes differ at {np.argwhere(pdiff)[:5].tolist()}"
            rep["pair_marginal"] = int(pm.sum())
    return rep


def compare_history(g, o, sc, dp, frac_eps=0.05, rel=1e-3, eps_abs=1e-4):
    """Per-iteration residual norms of the stopping test (Sec. V-A), device
    against oracle: |r_g - r_o| <= frac_eps * eps_pri + rel * r_o and the
    same for s, at every iteration both sides ran.  eps_pri is the run's own
    tolerance, and at least the absolute part of the workload's
    (sqrt(2 P T dp) eps_abs with eps_abs = 1e-4; sqrt(N T dp) eps_abs for s),
    so that a lockstep run with its tolerances set to zero keeps the same
    bar.  The stopping decision compares r with eps_pri, so an agreement to a
    small fraction of eps_pri makes the two decisions the same except at a
    near tie; FP32 positions of magnitude |p| carry an absolute rounding of
    about 6e-8 |p| per entry, far below 5% of eps_pri.  Returns the worst
    ratios."""
    K = min(len(g["hist"]), len(o["hist"]))
    assert K >= 1
    hg = np.asarray(g["hist"][:K], dtype=np.float64)
    ho = np.asarray(o["hist"][:K])
    P = sc.N * (sc.N - 1) / 2
    floor = {0: np.sqrt(2.0 * P * sc.T * dp) * eps_abs, 1: np.sqrt(float(sc.N) * sc.T * dp) * eps_abs}
    worst = [0.0, 0.0]
    for q, eps_col in ((0, 2), (1, 3)):
        bar = frac_eps * np.maximum(ho[:, eps_col], floor[q]) + rel * ho[:, q]
        ratio = np.abs(hg[:, q] - ho[:, q]) / bar
        worst[q] = float(ratio.max())
        bad = np.nonzero(ratio > 1.0)[0]
        assert bad.size == 0, (f"residual {'rs'[q]} differs at iteration {int(bad[0]) + 1}: "
                               f"gpu {hg[bad[0], q]:.6e} oracle {ho[bad[0], q]:.6e} eps {ho[bad[0], eps_col]:.3e}")
    return worst
