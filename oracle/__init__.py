"""FP64 reference ("oracle") for the ADMM multi-agent trajectory solver.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
path (the HIP library and its Python binding) never imports, links or calls it,
and it shares no code with that path: the two meet only in the seeded input
generators of ``synth``.

The numerical core is plain C (``tadmm_oracle.c``, FP64, OpenMP over agents or
scenarios); this module compiles it with gcc on first use and wraps it with
ctypes.  ``grad.py`` (the gradient through a converged solve, by the implicit
function theorem on the dense KKT system of its equality QP) is NumPy.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
import threading
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tadmm_oracle.c")
_HDR = os.path.join(_HERE, "tadmm_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CONVERGED, MAX_ITER, ACTIVE_SET_CAP, NONFINITE = 0, 1, 2, 3
NORMAL_PER_ITER, NORMAL_FROZEN = 0, 1
START_PREV, START_WARM, START_COLD = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the C oracle into oracle/liboracle.so (gcc -O3 -fopenmp).  The
    vector ISA is x86-64-v3 (AVX2, FMA) rather than the build host's own, so
    that the library also runs on another host; floating-point contraction
    is off, so every operation rounds as written."""
    stale = (not os.path.exists(_LIB) or
             os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(_HDR)))
    if force or stale:
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-std=c11", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fPIC", "-shared", "-fopenmp",
               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("nu", C.c_int), ("dp", C.c_int),
                ("A", C.c_double * 36), ("B", C.c_double * 18),
                ("u_lo", C.c_double * 3), ("u_hi", C.c_double * 3),
                ("qT_scale", C.c_double), ("d_min", C.c_double), ("rho", C.c_double),
                ("eps_abs", C.c_double), ("eps_rel", C.c_double), ("mu_tol", C.c_double),
                ("max_iter", C.c_int), ("max_as_iter", C.c_int), ("normal_mode", C.c_int),
                ("warm_start", C.c_int), ("hotstart", C.c_int), ("lu_reuse", C.c_int),
                ("fixed_iters", C.c_int), ("adaptive_rho", C.c_int), ("rho_mu", C.c_double),
                ("rho_tau", C.c_double), ("rho_every", C.c_int), ("state_box", C.c_int),
                ("s_lo", C.c_double * 3), ("s_hi", C.c_double * 3), ("p_lo", C.c_double * 3),
                ("p_hi", C.c_double * 3), ("alpha", C.c_double),
                ("momentum", C.c_int), ("mom_eta", C.c_double)]


_dp = C.POINTER(C.c_double)


class _Scenario(C.Structure):
    _fields_ = [("N", C.c_int), ("T", C.c_int), ("x0", _dp), ("xref", _dp),
                ("q_diag", _dp), ("r_diag", _dp), ("normals", _dp),
                ("agent_q", _dp), ("agent_r", _dp), ("agent_lo", _dp), ("agent_hi", _dp),
                ("agent_A", _dp), ("agent_B", _dp)]


class _Result(C.Structure):
    _fields_ = [("x", _dp), ("u", _dp), ("w", C.POINTER(C.c_byte)), ("mu", _dp),
                ("pair_active", C.POINTER(C.c_ubyte)), ("z", _dp), ("lam", _dp), ("hist", _dp),
                ("status", C.c_int), ("iters", C.c_int),
                ("r_norm", C.c_double), ("s_norm", C.c_double),
                ("eps_pri", C.c_double), ("eps_dual", C.c_double),
                ("as_passes", C.c_long), ("lu_factorizations", C.c_long), ("rho_hist", _dp)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            path = build()
            L = C.CDLL(path)
            L.orc_agent_qp.restype = C.c_int
            L.orc_agent_qp.argtypes = [C.POINTER(_Params), C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp,
                                       _dp, _dp, C.POINTER(C.c_byte), _dp, C.c_int,
                                       C.POINTER(C.c_long), C.POINTER(C.c_long)]
            L.orc_admm.restype = C.c_int
            L.orc_admm.argtypes = [C.POINTER(_Params), C.POINTER(_Scenario), C.POINTER(_Result), C.c_int]
            L.orc_admm_batch.restype = C.c_int
            L.orc_admm_batch.argtypes = [C.POINTER(_Params), C.c_int, C.POINTER(_Scenario),
                                         C.POINTER(_Result), C.c_int]
            L.orc_max_threads.restype = C.c_int
            L.orc_relinearize.restype = C.c_int
            L.orc_relinearize.argtypes = [C.POINTER(_Params), C.POINTER(_Scenario), _dp, _dp]
            _lib = L
    return _lib


def max_threads() -> int:
    return int(lib().orc_max_threads())


@dataclasses.dataclass
class OracleOptions:
    normal_mode: int = NORMAL_PER_ITER
    mu_tol: float = 1e-5
    max_as_iter: int = 0
    warm_start: bool = True
    hotstart: bool = True
    lu_reuse: bool = True
    fixed_iters: int = 0
    max_iter: Optional[int] = None   # None: the problem's max_iter
    eps_abs: Optional[float] = None
    eps_rel: Optional[float] = None
    rho: Optional[float] = None
    adaptive_rho: bool = False      # residual balancing (Boyd et al. 2011, Sec. 3.4.1)
    rho_mu: float = 10.0
    rho_tau: float = 2.0
    rho_every: int = 1
    state_box: bool = False         # box on the non-position states (a further ADMM split)
    s_lo: tuple = (-np.inf, -np.inf, -np.inf)
    s_hi: tuple = (np.inf, np.inf, np.inf)
    p_lo: tuple = (-np.inf, -np.inf, -np.inf)   # with state_box: the position box
    p_hi: tuple = (np.inf, np.inf, np.inf)
    alpha: float = 1.0              # over-relaxation (Boyd et al. 2011, Sec. 3.4.3)
    momentum: bool = False          # fast ADMM with restart (Goldstein et al. 2014, Alg. 8)
    mom_eta: float = 0.999


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return C.cast(None, _dp)
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def make_params(problem, opts: OracleOptions) -> _Params:
    p = _Params()
    nx, nu = problem.nx, problem.nu
    p.nx, p.nu, p.dp = nx, nu, problem.dp
    A, B = problem.A, problem.B
    for k, v in enumerate(A.reshape(-1)):
        p.A[k] = float(v)
    for k, v in enumerate(B.reshape(-1)):
        p.B[k] = float(v)
    for c in range(nu):
        p.u_lo[c] = float(problem.u_lo[c])
        p.u_hi[c] = float(problem.u_hi[c])
    p.qT_scale = float(problem.qT_scale)
    p.d_min = float(problem.d_min)
    p.rho = float(problem.rho if opts.rho is None else opts.rho)
    p.eps_abs = float(problem.eps_abs if opts.eps_abs is None else opts.eps_abs)
    p.eps_rel = float(problem.eps_rel if opts.eps_rel is None else opts.eps_rel)
    p.mu_tol = float(opts.mu_tol)
    p.max_iter = int(problem.max_iter if opts.max_iter is None else opts.max_iter)
    p.max_as_iter = int(opts.max_as_iter)
    p.normal_mode = int(opts.normal_mode)
    p.warm_start = int(bool(opts.warm_start))
    p.hotstart = int(bool(opts.hotstart))
    p.lu_reuse = int(bool(opts.lu_reuse))
    p.fixed_iters = int(opts.fixed_iters)
    p.adaptive_rho = int(bool(opts.adaptive_rho))
    p.rho_mu = float(opts.rho_mu)
    p.rho_tau = float(opts.rho_tau)
    p.rho_every = max(int(opts.rho_every), 1)
    p.state_box = int(bool(opts.state_box))
    for c in range(3):
        p.s_lo[c] = float(opts.s_lo[c])
        p.s_hi[c] = float(opts.s_hi[c])
        p.p_lo[c] = float(opts.p_lo[c])
        p.p_hi[c] = float(opts.p_hi[c])
    p.alpha = float(opts.alpha)
    p.momentum = int(bool(opts.momentum))
    p.mom_eta = float(opts.mom_eta)
    return p


class _Holder:
    """Keeps the numpy buffers of one scenario's inputs/outputs alive."""

    def __init__(self, problem, sc, opts: OracleOptions, normals=None, keep_zl=False, inputs=None):
        nx, nu, dp = problem.nx, problem.nu, problem.dp
        N, T = sc.N, sc.T
        P = N * (N - 1) // 2
        x0, xref = (sc.x0(), sc.xref()) if inputs is None else inputs
        self.x0 = np.ascontiguousarray(np.asarray(x0, dtype=np.float64).reshape(N, nx))
        self.xref = np.ascontiguousarray(np.asarray(xref, dtype=np.float64).reshape(N, T + 1, nx))
        self.q = np.ascontiguousarray(problem.q_diag if sc.q_diag is None else sc.q_diag, dtype=np.float64)
        self.r = np.ascontiguousarray(problem.r_diag if sc.r_diag is None else sc.r_diag, dtype=np.float64)
        self.normals = None if normals is None else np.ascontiguousarray(normals, dtype=np.float64).reshape(P, T, dp)
        maxit = opts.fixed_iters if opts.fixed_iters > 0 else (problem.max_iter if opts.max_iter is None else opts.max_iter)
        self.x = np.zeros((N, T + 1, nx))
        self.u = np.zeros((N, T, nu))
        self.w = np.zeros((N, T, nu), dtype=np.int8)
        self.mu = np.zeros((N, T, nu))
        self.pa = np.zeros((P, T), dtype=np.uint8)
        self.hist = np.zeros((max(maxit, 1), 4))
        self.rho_hist = np.zeros(max(maxit, 1))
        self.z = np.zeros((N, N, T, dp)) if keep_zl else None
        self.lam = np.zeros((N, N, T, dp)) if keep_zl else None
        # heterogeneous agents: per-agent weights, input boxes, dynamics (optional)
        per = lambda f, w: (None if getattr(sc, f, None) is None else
                            np.ascontiguousarray(np.asarray(getattr(sc, f), dtype=np.float64).reshape(N, w)))
        self.aq, self.ar = per("agent_q", nx), per("agent_r", nu)
        self.alo, self.ahi = per("agent_lo", nu), per("agent_hi", nu)
        self.aA, self.aB = per("agent_A", nx * nx), per("agent_B", nx * nu)
        self.sc = _Scenario(N, T, _ptr(self.x0), _ptr(self.xref), _ptr(self.q), _ptr(self.r), _ptr(self.normals),
                            _ptr(self.aq), _ptr(self.ar), _ptr(self.alo), _ptr(self.ahi), _ptr(self.aA),
                            _ptr(self.aB))
        self.res = _Result(_ptr(self.x), _ptr(self.u), self.w.ctypes.data_as(C.POINTER(C.c_byte)), _ptr(self.mu),
                           self.pa.ctypes.data_as(C.POINTER(C.c_ubyte)), _ptr(self.z), _ptr(self.lam),
                           _ptr(self.hist), 0, 0, 0.0, 0.0, 0.0, 0.0, 0, 0, _ptr(self.rho_hist))

    def output(self) -> Dict[str, object]:
        r = self.res
        out = dict(x=self.x, u=self.u, w=self.w, mu=self.mu, pair_active=self.pa,
                   status=int(r.status), iters=int(r.iters), r_norm=float(r.r_norm), s_norm=float(r.s_norm),
                   eps_pri=float(r.eps_pri), eps_dual=float(r.eps_dual), as_passes=int(r.as_passes),
                   lu_factorizations=int(r.lu_factorizations), hist=self.hist[:max(int(r.iters), 0)],
                   rho_hist=self.rho_hist[:max(int(r.iters), 0)])
        if self.z is not None:
            out["z"] = self.z
            out["lam"] = self.lam
        return out


def solve(problem, scenario, opts: Optional[OracleOptions] = None, normals=None, threads: int = 1,
          keep_zl: bool = False, inputs=None) -> Dict[str, object]:
    """ADMM on one scenario.  Returns numpy arrays x [N][T+1][nx], u [N][T][nu],
    w [N][T][nu] (0 free / 1 lower / 2 upper), mu, pair_active [P][T], and the
    status, iteration count and final residuals.  `inputs` = (x0, xref)
    replaces the scenario's own initial states and references."""
    opts = opts or OracleOptions()
    prm = make_params(problem, opts)
    h = _Holder(problem, scenario, opts, normals, keep_zl, inputs)
    rc = lib().orc_admm(C.byref(prm), C.byref(h.sc), C.byref(h.res), int(threads))
    if rc != 0:
        raise RuntimeError("oracle ADMM failed (allocation or singular KKT)")
    return h.output()


def solve_batch(problem, scenarios: Sequence, opts: Optional[OracleOptions] = None, threads: int = 0,
                normals: Optional[List[np.ndarray]] = None, inputs=None,
                keep_zl: bool = False) -> List[Dict[str, object]]:
    """Independent scenarios, OpenMP over scenarios (dynamic schedule).
    keep_zl: also return the consensus copies z and duals lambda."""
    opts = opts or OracleOptions()
    prm = make_params(problem, opts)
    hs = [_Holder(problem, sc, opts, None if normals is None else normals[k], keep_zl,
                  None if inputs is None else inputs[k]) for k, sc in enumerate(scenarios)]
    S = len(hs)
    scs = (_Scenario * max(S, 1))(*[h.sc for h in hs])
    res = (_Result * max(S, 1))(*[h.res for h in hs])
    th = threads if threads > 0 else max_threads()
    rc = lib().orc_admm_batch(C.byref(prm), S, scs, res, int(th))
    if rc != 0:
        raise RuntimeError("oracle batch failed")
    for k, h in enumerate(hs):
        h.res = res[k]
    return [h.output() for h in hs]


def agent_qp(problem, T: int, n_nbr: int, x0, xref, q_diag, r_diag, ysum=None, start: int = START_WARM,
             x=None, u=None, w=None, opts: Optional[OracleOptions] = None) -> Dict[str, object]:
    """One agent's local QP (Eq. 3) with the consensus data folded into
    ysum[t] = sum_j (rho z_ij,t - lambda_ij,t) (t = 1..T; row 0 ignored)."""
    opts = opts or OracleOptions()
    prm = make_params(problem, opts)
    nx, nu, dp = problem.nx, problem.nu, problem.dp
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    xref = np.ascontiguousarray(xref, dtype=np.float64).reshape(T + 1, nx)
    q = np.ascontiguousarray(q_diag, dtype=np.float64)
    r = np.ascontiguousarray(r_diag, dtype=np.float64)
    ys = None if ysum is None else np.ascontiguousarray(ysum, dtype=np.float64).reshape(T + 1, dp)
    X = np.zeros((T + 1, nx)) if x is None else np.array(x, dtype=np.float64).reshape(T + 1, nx)
    U = np.zeros((T, nu)) if u is None else np.array(u, dtype=np.float64).reshape(T, nu)
    Wb = np.zeros((T, nu), dtype=np.int8) if w is None else np.array(w, dtype=np.int8).reshape(T, nu)
    mu = np.zeros((T, nu))
    passes, facts = C.c_long(0), C.c_long(0)
    rc = lib().orc_agent_qp(C.byref(prm), int(T), int(n_nbr), _ptr(x0), _ptr(xref), _ptr(q), _ptr(r), _ptr(ys),
                            _ptr(X), _ptr(U), Wb.ctypes.data_as(C.POINTER(C.c_byte)), _ptr(mu), int(start),
                            C.byref(passes), C.byref(facts))
    if rc < 0:
        raise RuntimeError("oracle agent QP failed")
    return dict(x=X, u=U, w=Wb, mu=mu, capped=(rc == 1), passes=int(passes.value), facts=int(facts.value))


def relinearize(problem, scenario, x, inputs=None) -> np.ndarray:
    """Normals [P][T][dp] of every pair (i < j) and step t = 1..T linearized
    about the positions of x [N][T+1][nx] (the reference normal where two
    positions coincide)."""
    opts = OracleOptions(normal_mode=NORMAL_FROZEN)
    prm = make_params(problem, opts)
    h = _Holder(problem, scenario, opts, None, False, inputs)
    N, T, dp = scenario.N, scenario.T, problem.dp
    xx = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(N, T + 1, problem.nx))
    out = np.zeros((N * (N - 1) // 2, T, dp))
    rc = lib().orc_relinearize(C.byref(prm), C.byref(h.sc), _ptr(xx), _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle relinearize failed")
    return out
