"""MI355X (gfx950) ADMM multi-agent trajectory solver -- Python binding.

Thin ctypes layer over ``libturboadmm.so`` (C ABI in ``include/turboadmm.h``).
Every step of the solve runs in the HIP kernels of that library; this module
only marshals arguments.  PyTorch supplies device memory and the stream.
There is no CPU fallback: if the library is missing, the import of the
binding raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libturboadmm.so")

OK = 0
STATUS_NAMES = {0: "ok", 1: "invalid argument", 2: "shape error", 3: "non-finite input", 4: "infeasible start",
                5: "HIP runtime error", 6: "workspace error", 7: "state error"}
SCEN_CONVERGED, SCEN_MAX_ITER, SCEN_ACTIVE_SET_CAP, SCEN_NONFINITE = 0, 1, 2, 3
NORMAL_PER_ITER, NORMAL_FROZEN = 0, 1
MODE_PLAIN, MODE_BATCHED, MODE_WIDE = 0, 1, 2


class TadmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"turboadmm error {code} ({STATUS_NAMES.get(code, '?')}): {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nu", C.c_int32),
                ("A", C.c_float * 36), ("B", C.c_float * 18),
                ("u_lo", C.c_float * 3), ("u_hi", C.c_float * 3),
                ("qT_scale", C.c_float), ("d_min", C.c_float), ("rho", C.c_float),
                ("eps_abs", C.c_float), ("eps_rel", C.c_float), ("mu_tol", C.c_float),
                ("max_iter", C.c_int32), ("max_as_iter", C.c_int32), ("normal_mode", C.c_int32),
                ("cache_factors", C.c_int32), ("riccati_warmstart", C.c_int32), ("hotstart", C.c_int32),
                ("check_inputs", C.c_int32), ("block_threads", C.c_int32), ("refine", C.c_int32),
                ("refine_band", C.c_float), ("eqp_fp64", C.c_int32), ("adaptive_rho", C.c_int32),
                ("rho_mu", C.c_float), ("rho_tau", C.c_float), ("rho_every", C.c_int32),
                ("state_box", C.c_int32), ("s_lo", C.c_float * 3), ("s_hi", C.c_float * 3),
                ("alpha", C.c_float), ("p_lo", C.c_float * 3), ("p_hi", C.c_float * 3),
                ("momentum", C.c_int32), ("mom_eta", C.c_float)]


_fp = C.POINTER(C.c_float)
_ip = C.POINTER(C.c_int32)


class Batch(C.Structure):
    _fields_ = [("n_scen", C.c_int32), ("n_agents", _ip), ("horizon", _ip),
                ("x0", C.c_void_p), ("xref", C.c_void_p), ("q_diag", C.c_void_p), ("r_diag", C.c_void_p),
                ("normals", C.c_void_p), ("agent_q", C.c_void_p), ("agent_r", C.c_void_p),
                ("agent_lo", C.c_void_p), ("agent_hi", C.c_void_p), ("agent_A", C.c_void_p), ("agent_B", C.c_void_p)]


class Out(C.Structure):
    _fields_ = [("x", C.c_void_p), ("u", C.c_void_p), ("w", C.c_void_p), ("pair_active", C.c_void_p),
                ("status", C.c_void_p), ("iters", C.c_void_p), ("r_norm", C.c_void_p), ("s_norm", C.c_void_p),
                ("eps_pri", C.c_void_p), ("eps_dual", C.c_void_p), ("counters", C.c_void_p),
                ("hist", C.c_void_p)]


_lib = None


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.tadmm_workspace_size.restype = C.c_int
        L.tadmm_workspace_size.argtypes = [C.POINTER(Params), C.c_int32, _ip, _ip, C.POINTER(C.c_size_t)]
        L.tadmm_create.restype = C.c_int
        L.tadmm_create.argtypes = [C.POINTER(vp), C.POINTER(Params), vp]
        L.tadmm_solve.restype = C.c_int
        L.tadmm_solve.argtypes = [vp, C.POINTER(Batch), C.POINTER(Out), vp, C.c_size_t, C.c_int32]
        L.tadmm_solve_noalloc.restype = C.c_int
        L.tadmm_solve_noalloc.argtypes = [vp, C.POINTER(Batch), C.POINTER(Out), C.c_int32]
        L.tadmm_polish.restype = C.c_int
        L.tadmm_polish.argtypes = [vp, C.POINTER(Batch), C.POINTER(Out), vp, C.c_size_t, vp]
        L.tadmm_adjoint.restype = C.c_int
        L.tadmm_adjoint.argtypes = [vp, C.POINTER(Batch), C.POINTER(Out), vp, C.c_size_t, vp, vp, vp, vp, vp, vp, vp]
        L.tadmm_sqp.restype = C.c_int
        L.tadmm_sqp.argtypes = [vp, C.POINTER(Batch), C.POINTER(Out), vp, C.c_size_t, C.c_int32, C.c_int32,
                                C.c_float, C.c_float, vp]
        L.tadmm_autotune.restype = C.c_int
        L.tadmm_autotune.argtypes = [vp, C.POINTER(Batch), C.POINTER(Out), vp, C.c_size_t, _ip]
        L.tadmm_last_kernel_ms.restype = C.c_float
        L.tadmm_last_kernel_ms.argtypes = [vp]
        L.tadmm_destroy.restype = C.c_int
        L.tadmm_destroy.argtypes = [vp]
        L.tadmm_status_string.restype = C.c_char_p
        L.tadmm_status_string.argtypes = [C.c_int]
        L.tadmm_last_error.restype = C.c_char_p
        L.tadmm_last_error.argtypes = [vp]
        L.tadmm_version.restype = C.c_char_p
        L.tadmm_version.argtypes = []
        _lib = L
    return _lib


EXPORTED_SYMBOLS = ("tadmm_workspace_size", "tadmm_create", "tadmm_solve", "tadmm_solve_noalloc", "tadmm_sqp",
                    "tadmm_polish",
                    "tadmm_adjoint", "tadmm_autotune",
                    "tadmm_last_kernel_ms", "tadmm_destroy", "tadmm_status_string", "tadmm_last_error",
                    "tadmm_version")


def make_params(problem, *, normal_mode: int = NORMAL_PER_ITER, mu_tol: float = 1e-5, max_as_iter: int = 0,
                cache_factors: bool = True, riccati_warmstart: bool = True, hotstart: bool = True,
                check_inputs: bool = True, block_threads: int = 0, refine: bool = True,
                refine_band: float = 10.0, eqp_fp64: bool = True, adaptive_rho: bool = False,
                rho_mu: float = 10.0, rho_tau: float = 2.0, rho_every: int = 1, state_box: bool = False,
                s_lo: Optional[Sequence[float]] = None, s_hi: Optional[Sequence[float]] = None,
                alpha: float = 1.0, p_lo: Optional[Sequence[float]] = None,
                p_hi: Optional[Sequence[float]] = None, momentum: bool = False, mom_eta: float = 0.999,
                max_iter: Optional[int] = None,
                eps_abs: Optional[float] = None, eps_rel: Optional[float] = None,
                rho: Optional[float] = None) -> Params:
    """Fill the C parameter struct from a problem description (attributes
    nx, nu, A, B, u_lo, u_hi, qT_scale, d_min, rho, eps_abs, eps_rel,
    max_iter, e.g. ``synth.ProblemParams``)."""
    p = Params()
    p.nx, p.nu = int(problem.nx), int(problem.nu)
    for k, v in enumerate(np.asarray(problem.A, dtype=np.float64).reshape(-1)):
        p.A[k] = float(v)
    for k, v in enumerate(np.asarray(problem.B, dtype=np.float64).reshape(-1)):
        p.B[k] = float(v)
    for c in range(p.nu):
        p.u_lo[c] = float(problem.u_lo[c])
        p.u_hi[c] = float(problem.u_hi[c])
    p.qT_scale = float(problem.qT_scale)
    p.d_min = float(problem.d_min)
    p.rho = float(problem.rho if rho is None else rho)
    p.eps_abs = float(problem.eps_abs if eps_abs is None else eps_abs)
    p.eps_rel = float(problem.eps_rel if eps_rel is None else eps_rel)
    p.mu_tol = float(mu_tol)
    p.max_iter = int(problem.max_iter if max_iter is None else max_iter)
    p.max_as_iter = int(max_as_iter)
    p.normal_mode = int(normal_mode)
    p.cache_factors = int(bool(cache_factors))
    p.riccati_warmstart = int(bool(riccati_warmstart))
    p.hotstart = int(bool(hotstart))
    p.check_inputs = int(bool(check_inputs))
    p.block_threads = int(block_threads)
    p.refine = int(bool(refine))
    p.refine_band = float(refine_band)
    p.eqp_fp64 = int(bool(eqp_fp64))
    p.adaptive_rho = int(bool(adaptive_rho))
    p.rho_mu = float(rho_mu)
    p.rho_tau = float(rho_tau)
    p.rho_every = int(rho_every)
    p.state_box = int(bool(state_box))
    for c in range(3):
        p.s_lo[c] = float(-np.inf if s_lo is None or c >= len(s_lo) else s_lo[c])
        p.s_hi[c] = float(np.inf if s_hi is None or c >= len(s_hi) else s_hi[c])
    p.alpha = float(alpha)
    for c in range(3):
        p.p_lo[c] = float(-np.inf if p_lo is None or c >= len(p_lo) else p_lo[c])
        p.p_hi[c] = float(np.inf if p_hi is None or c >= len(p_hi) else p_hi[c])
    p.momentum = int(bool(momentum))
    p.mom_eta = float(mom_eta)
    return p


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Solver:
    """One context of the C library, bound to a torch device and stream."""

    def __init__(self, params: Params, device=None, stream=None):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.params = params
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
            h = C.c_void_p()
            rc = lib().tadmm_create(C.byref(h), C.byref(params), C.c_void_p(self.stream.cuda_stream))
        if rc != OK:
            raise TadmmError(rc, "tadmm_create failed")
        self._h = h
        self._ws = None

    def close(self):
        if getattr(self, "_h", None):
            lib().tadmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != OK:
            raise TadmmError(rc, lib().tadmm_last_error(self._h).decode())

    def workspace_bytes(self, n_agents: np.ndarray, horizon: np.ndarray) -> int:
        nb = C.c_size_t(0)
        N = np.ascontiguousarray(n_agents, dtype=np.int32)
        T = np.ascontiguousarray(horizon, dtype=np.int32)
        rc = lib().tadmm_workspace_size(C.byref(self.params), int(N.size), N.ctypes.data_as(_ip),
                                        T.ctypes.data_as(_ip), C.byref(nb))
        if rc != OK:
            raise TadmmError(rc, "tadmm_workspace_size failed")
        return int(nb.value)

    def prepare(self, n_agents, horizon, x0, xref, q_diag, r_diag, normals=None, agent_q=None, agent_r=None,
                agent_lo=None, agent_hi=None, agent_A=None, agent_B=None, history: bool = False):
        """Allocate device inputs, outputs and the workspace for a batch.
        agent_q [A][nx], agent_r [A][nu], agent_lo / agent_hi [A][nu],
        agent_A [A][nx*nx], agent_B [A][nx*nu]: heterogeneous agents (each
        optional).  history: also record the residual norms of every
        iteration (output "hist" [S][max_iter][2])."""
        torch = self.torch
        N = np.ascontiguousarray(n_agents, dtype=np.int32)
        T = np.ascontiguousarray(horizon, dtype=np.int32)
        nx, nu = self.params.nx, self.params.nu
        dev = self.device

        def dt(a, shape):
            t = torch.as_tensor(np.asarray(a, dtype=np.float32) if not torch.is_tensor(a) else a)
            return t.to(device=dev, dtype=torch.float32).contiguous().reshape(shape)

        S = int(N.size)
        A = int(N.sum())
        GS = int((N * (T + 1)).sum())
        GU = int((N * T).sum())
        PT = int((N * (N - 1) // 2 * T).sum())
        b = dict(N=N, T=T,
                 x0=dt(x0, (A, nx)), xref=dt(xref, (GS, nx)),
                 q_diag=dt(q_diag, (S, nx)), r_diag=dt(r_diag, (S, nu)),
                 normals=None if normals is None else dt(normals, (PT, nu)),
                 agent_q=None if agent_q is None else dt(agent_q, (A, nx)),
                 agent_r=None if agent_r is None else dt(agent_r, (A, nu)),
                 agent_lo=None if agent_lo is None else dt(agent_lo, (A, nu)),
                 agent_hi=None if agent_hi is None else dt(agent_hi, (A, nu)),
                 agent_A=None if agent_A is None else dt(agent_A, (A, nx * nx)),
                 agent_B=None if agent_B is None else dt(agent_B, (A, nx * nu)))
        o = dict(x=torch.zeros(GS, nx, device=dev), u=torch.zeros(GU, nu, device=dev),
                 w=torch.zeros(GU, nu, dtype=torch.int8, device=dev),
                 pair_active=torch.zeros(PT, dtype=torch.uint8, device=dev),
                 status=torch.zeros(S, dtype=torch.int32, device=dev), iters=torch.zeros(S, dtype=torch.int32, device=dev),
                 r_norm=torch.zeros(S, device=dev), s_norm=torch.zeros(S, device=dev),
                 eps_pri=torch.zeros(S, device=dev), eps_dual=torch.zeros(S, device=dev),
                 counters=torch.zeros(S, 8, dtype=torch.int64, device=dev),
                 hist=(torch.zeros(S, int(self.params.max_iter), 2, device=dev) if history else None))
        nbytes = self.workspace_bytes(N, T)
        ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        return Prepared(self, b, o, ws, nbytes)

    def solve(self, n_agents, horizon, x0, xref, q_diag, r_diag, normals=None, mode: int = MODE_BATCHED) -> Dict:
        prep = self.prepare(n_agents, horizon, x0, xref, q_diag, r_diag, normals)
        prep.run(mode)
        return prep.result()


class Prepared:
    """A batch resident on the device, with its outputs and workspace; `run`
    can be called repeatedly (the timed region of the benchmark)."""

    def __init__(self, solver: Solver, b: Dict, o: Dict, ws, nbytes: int):
        self.solver, self.b, self.o, self.ws, self.nbytes = solver, b, o, ws, nbytes
        self.batch = Batch(int(b["N"].size), b["N"].ctypes.data_as(_ip), b["T"].ctypes.data_as(_ip),
                           _ptr(b["x0"]), _ptr(b["xref"]), _ptr(b["q_diag"]), _ptr(b["r_diag"]), _ptr(b["normals"]),
                           _ptr(b["agent_q"]), _ptr(b["agent_r"]), _ptr(b["agent_lo"]), _ptr(b["agent_hi"]),
                           _ptr(b["agent_A"]), _ptr(b["agent_B"]))
        self.out = Out(*[_ptr(o[k]) for k in ("x", "u", "w", "pair_active", "status", "iters", "r_norm", "s_norm",
                                              "eps_pri", "eps_dual", "counters", "hist")])

    def run(self, mode: int = MODE_BATCHED):
        s = self.solver
        rc = lib().tadmm_solve(s._h, C.byref(self.batch), C.byref(self.out), C.c_void_p(self.ws.data_ptr()),
                               C.c_size_t(self.nbytes), int(mode))
        s._check(rc)
        return lib().tadmm_last_kernel_ms(s._h)

    def run_noalloc(self, mode: int = MODE_BATCHED):
        """The same solve through tadmm_solve_noalloc (the library's static
        workspace instead of self.ws; nothing is allocated by the call)."""
        s = self.solver
        rc = lib().tadmm_solve_noalloc(s._h, C.byref(self.batch), C.byref(self.out), int(mode))
        s._check(rc)
        return lib().tadmm_last_kernel_ms(s._h)

    def sqp(self, mode: int = MODE_BATCHED, max_rounds: int = 10, rtol: float = 1e-4, sep_tol: float = 1e-2):
        """SQP outer loop (tadmm_sqp): rounds of frozen-normal solves,
        re-linearized about each solution.  Returns the per-scenario stats
        [S][4]: rounds, stopping rule met, objective, smallest distance."""
        torch = self.solver.torch
        s = self.solver
        st = torch.zeros(self.b["N"].size, 4, device=s.device)
        rc = lib().tadmm_sqp(s._h, C.byref(self.batch), C.byref(self.out), C.c_void_p(self.ws.data_ptr()),
                             C.c_size_t(self.nbytes), int(mode), int(max_rounds), float(rtol), float(sep_tol), _ptr(st))
        s._check(rc)
        return st

    def autotune(self) -> int:
        s = self.solver
        best = C.c_int32(0)
        rc = lib().tadmm_autotune(s._h, C.byref(self.batch), C.byref(self.out), C.c_void_p(self.ws.data_ptr()),
                                  C.c_size_t(self.nbytes), C.byref(best))
        s._check(rc)
        return int(best.value)

    def polish(self):
        """Replace the solution of the last run with the solution of its
        equality QP (tadmm_polish); returns the per-scenario stats [S][4]."""
        torch = self.solver.torch
        s = self.solver
        st = torch.zeros(self.b["N"].size, 4, device=s.device)
        rc = lib().tadmm_polish(s._h, C.byref(self.batch), C.byref(self.out), C.c_void_p(self.ws.data_ptr()),
                                C.c_size_t(self.nbytes), _ptr(st))
        s._check(rc)
        return st

    def adjoint(self, dL_dx, dL_du=None, want_stats: bool = False):
        """Gradients of a loss through the polished solution (tadmm_adjoint).
        Returns (dL_dx0, dL_dxref, dL_dlogq, dL_dlogr) [, stats]."""
        torch = self.solver.torch
        s, b = self.solver, self.b
        dev = s.device
        gx = dL_dx.to(device=dev, dtype=torch.float32).contiguous()
        gu = None if dL_du is None else dL_du.to(device=dev, dtype=torch.float32).contiguous()
        outs = (torch.zeros_like(b["x0"]), torch.zeros_like(b["xref"]), torch.zeros_like(b["q_diag"]),
                torch.zeros_like(b["r_diag"]))
        st = torch.zeros(b["N"].size, 4, device=dev)
        rc = lib().tadmm_adjoint(s._h, C.byref(self.batch), C.byref(self.out), C.c_void_p(self.ws.data_ptr()),
                                 C.c_size_t(self.nbytes), _ptr(gx), _ptr(gu), *[_ptr(t) for t in outs], _ptr(st))
        s._check(rc)
        return (outs + (st,)) if want_stats else outs

    def result(self) -> Dict:
        r = dict(self.o)
        r["kernel_ms"] = lib().tadmm_last_kernel_ms(self.solver._h)
        return r


def straight_line_ref(starts, goals, T: int, dt: float):
    """Constant-velocity references from rest positions to goals, as torch
    ops (so that gradients reach the goals): r_t = (p_s + (t/T)(g - p_s),
    (g - p_s)/(T dt)), t = 0..T.  starts, goals [N][dp] -> [N][T+1][2 dp]."""
    import torch
    frac = torch.arange(T + 1, device=starts.device, dtype=starts.dtype) / T
    d = goals - starts
    pos = starts[:, None, :] + frac[None, :, None] * d[:, None, :]
    vel = (d / (T * dt))[:, None, :].expand(-1, T + 1, -1)
    return torch.cat([pos, vel], dim=2)


def _autograd_function():
    import torch

    class TurboADMMFunction(torch.autograd.Function):
        """(x, u) = argmin of the batch (tadmm_solve + tadmm_polish); the
        backward pass is tadmm_adjoint.  Arguments: x0 [sum N][nx], xref
        [sum N (T+1)][nx], log_q [S][nx], log_r [S][nu] (device tensors) and a
        config dict with keys solver (Solver), n_agents, horizon and optional
        normals and mode.  After the call, config["prepared"] holds the batch
        (statuses, iteration counts, polish statistics)."""

        @staticmethod
        def forward(ctx, x0, xref, log_q, log_r, config):
            solver = config["solver"]
            prep = solver.prepare(config["n_agents"], config["horizon"], x0.detach(), xref.detach(),
                                  torch.exp(log_q.detach()), torch.exp(log_r.detach()), config.get("normals"))
            prep.run(config.get("mode", MODE_BATCHED))
            prep.polish_stats = prep.polish()
            config["prepared"] = prep
            ctx.prep = prep
            return prep.o["x"].clone(), prep.o["u"].clone()

        @staticmethod
        def backward(ctx, gx, gu):
            dx0, dxref, dlogq, dlogr = ctx.prep.adjoint(gx, gu)
            return dx0, dxref, dlogq, dlogr, None

    return TurboADMMFunction


class _Lazy:
    """Creates the autograd Function on first use (torch is imported lazily)."""
    _fn = None

    def __getattr__(self, name):
        if _Lazy._fn is None:
            _Lazy._fn = _autograd_function()
        return getattr(_Lazy._fn, name)


TurboADMMFunction = _Lazy()


def split_outputs(res: Dict, n_agents: Sequence[int], horizon: Sequence[int], nx: int, nu: int):
    """Per-scenario numpy views of a result: list of dicts with x [N][T+1][nx],
    u [N][T][nu], w, pair_active [P][T], status, iters."""
    host = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items() if v is not None}
    out = []
    xo = uo = po = 0
    for s, (N, T) in enumerate(zip(n_agents, horizon)):
        N, T = int(N), int(T)
        P = N * (N - 1) // 2
        d = dict(x=host["x"][xo:xo + N * (T + 1)].reshape(N, T + 1, nx),
                 u=host["u"][uo:uo + N * T].reshape(N, T, nu),
                 w=host["w"][uo:uo + N * T].reshape(N, T, nu),
                 pair_active=host["pair_active"][po:po + P * T].reshape(P, T),
                 status=int(host["status"][s]), iters=int(host["iters"][s]),
                 r_norm=float(host["r_norm"][s]), s_norm=float(host["s_norm"][s]),
                 eps_pri=float(host["eps_pri"][s]), eps_dual=float(host["eps_dual"][s]),
                 counters=host["counters"][s])
        if "hist" in host:
            d["hist"] = host["hist"][s, :d["iters"]]
        out.append(d)
        xo += N * (T + 1)
        uo += N * T
        po += P * T
    return out
