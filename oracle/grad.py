"""FP64 reference gradients through a converged solve (TEST INFRASTRUCTURE).

Only the test suite may import this module; the product path never does.

The converged solution is treated as the solution of the centralized QP of
Sec. III-A (Eq. 1) with its final active sets held as equalities: the input
bounds of the working sets W, and the binding separation half-planes A_c with
their normals n held constant (Eq. 4 with the linearization frozen).  That
equality QP (EQP)

    min_w 1/2 w'H(theta) w + c(theta)'w   s.t.  E w = e(theta)

has the KKT map F(w, y; theta) = [H w + c + E'y ; E w - e] = 0, and by the
implicit function theorem the gradient of a loss L(w) is

    dL/dtheta = -[wbar; ybar]' dF/dtheta,   K [wbar; ybar] = [dL/dw; 0],

with K the (symmetric) KKT matrix.  Here K is assembled densely and the
partial derivatives dF/dtheta are written out in closed form (only H, c and
e depend on theta; see implicit_gradient), everything in FP64.  A second,
independent reference re-solves the EQP at theta +- h (central finite
differences of the whole solve).

Parameters theta: the log of the diagonal of Q (nx), the log of the diagonal
of R (nu), the initial states x0 [N][nx] and the references xref [N][T+1][nx].
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg as sla

PARAMS = ("logq", "logr", "x0", "xref")


@dataclasses.dataclass
class EqpInstance:
    """One scenario's EQP: problem constants, data and the frozen active sets."""
    A: np.ndarray            # [nx][nx]
    B: np.ndarray            # [nx][nu]
    u_lo: np.ndarray         # [nu]
    u_hi: np.ndarray         # [nu]
    qT_scale: float
    d_min: float
    x0: np.ndarray           # [N][nx]
    xref: np.ndarray         # [N][T+1][nx]
    logq: np.ndarray         # [nx]
    logr: np.ndarray         # [nu]
    W: np.ndarray            # [N][T][nu]  0 free, 1 lower, 2 upper
    active: List[Tuple[int, int, int]]   # binding half-planes (i, j, t), i < j, t = 1..T
    normals: Dict[Tuple[int, int, int], np.ndarray]   # n for every pair-step (i, j, t)

    @property
    def N(self):
        return self.x0.shape[0]

    @property
    def T(self):
        return self.xref.shape[1] - 1

    @property
    def nx(self):
        return self.A.shape[0]

    @property
    def nu(self):
        return self.B.shape[1]

    def theta(self) -> Dict[str, np.ndarray]:
        return dict(logq=self.logq.copy(), logr=self.logr.copy(), x0=self.x0.copy(), xref=self.xref.copy())


def _layout(ins: EqpInstance):
    """Variable order: per agent, u_0..u_{T-1} then x_1..x_T."""
    N, T, nx, nu = ins.N, ins.T, ins.nx, ins.nu
    per = T * (nu + nx)
    iu = lambda i, t, c: i * per + t * nu + c
    ix = lambda i, t, r: i * per + T * nu + (t - 1) * nx + r   # t = 1..T
    return N * per, iu, ix


def constraints(ins: EqpInstance):
    """E and the row tags of the EQP; E does not depend on theta.

    Rows: for every agent the dynamics x_{t+1} - A x_t - B u_t = (A x0 at
    t = 0, else 0), then its inputs in W at their bounds; then one row
    n'(C x_i,t - C x_j,t) = d_min per half-plane of A_c (C picks the first
    dp = nu state components, the positions)."""
    N, T, nx, nu = ins.N, ins.T, ins.nx, ins.nu
    n, iu, ix = _layout(ins)
    rows, tags = [], []
    for i in range(N):
        for t in range(T):
            for k in range(nx):
                row = np.zeros(n)
                row[ix(i, t + 1, k)] = 1.0
                if t >= 1:
                    for m in range(nx):
                        row[ix(i, t, m)] -= ins.A[k, m]
                for a in range(nu):
                    row[iu(i, t, a)] -= ins.B[k, a]
                rows.append(row)
                tags.append(("dyn", i, t, k))
        for t in range(T):
            for a in range(nu):
                if ins.W[i, t, a]:
                    row = np.zeros(n)
                    row[iu(i, t, a)] = 1.0
                    rows.append(row)
                    tags.append(("bound", i, t, a))
    for (i, j, t) in ins.active:
        nv = ins.normals[(i, j, t)]
        row = np.zeros(n)
        for k in range(nu):
            row[ix(i, t, k)] += nv[k]
            row[ix(j, t, k)] -= nv[k]
        rows.append(row)
        tags.append(("pair", i, j, t))
    return np.array(rows).reshape(len(rows), n), tags


def objective(ins: EqpInstance, theta: Optional[Dict[str, np.ndarray]] = None):
    """Diagonal H and linear term c of the EQP cost.

    Cost (Eq. 1, no 1/2): sum_t (x_t - r_t)'Q_t(x_t - r_t) + u_t'R u_t with
    Q_t = Q for t < T and qT_scale Q at t = T; the t = 0 state term is a
    constant.  So H = 2 Q_t on x_t, 2 R on u_t and c = -2 Q_t r_t."""
    th = ins.theta() if theta is None else theta
    q, r = np.exp(th["logq"]), np.exp(th["logr"])
    xref = th["xref"]
    N, T, nx, nu = ins.N, ins.T, ins.nx, ins.nu
    n, iu, ix = _layout(ins)
    H = np.zeros(n)
    c = np.zeros(n)
    for i in range(N):
        H[iu(i, 0, 0):iu(i, 0, 0) + T * nu] = np.tile(2.0 * r, T)
        for t in range(1, T + 1):
            w = ins.qT_scale if t == T else 1.0
            s = ix(i, t, 0)
            H[s:s + nx] = 2.0 * w * q
            c[s:s + nx] = -2.0 * w * q * xref[i, t]
    return H, c


def rhs(ins: EqpInstance, tags, theta: Optional[Dict[str, np.ndarray]] = None):
    """e of E w = e: A x0 on the first dynamics rows, the bound values, d_min."""
    th = ins.theta() if theta is None else theta
    x0 = th["x0"]
    e = np.zeros(len(tags))
    for k, tg in enumerate(tags):
        if tg[0] == "dyn":
            _, i, t, r = tg
            e[k] = float(ins.A[r] @ x0[i]) if t == 0 else 0.0
        elif tg[0] == "bound":
            _, i, t, a = tg
            e[k] = ins.u_lo[a] if ins.W[i, t, a] == 1 else ins.u_hi[a]
        else:
            e[k] = ins.d_min
    return e


def kkt_matrix(H, E):
    n, m = H.size, E.shape[0]
    K = np.zeros((n + m, n + m))
    K[:n, :n] = np.diag(H)
    K[:n, n:] = E.T
    K[n:, :n] = E
    return K


def solve(ins: EqpInstance, theta=None, E=None, tags=None):
    """EQP solution (w, y) by one dense KKT solve."""
    if E is None:
        E, tags = constraints(ins)
    H, c = objective(ins, theta)
    sol = np.linalg.solve(kkt_matrix(H, E), np.concatenate([-c, rhs(ins, tags, theta)]))
    return sol[:H.size], sol[H.size:]


def trajectories(ins: EqpInstance, w, theta=None):
    """Unpack w into x [N][T+1][nx] (x_0 = x0) and u [N][T][nu]."""
    x0 = ins.x0 if theta is None else theta["x0"]
    N, T, nx, nu = ins.N, ins.T, ins.nx, ins.nu
    per = T * (nu + nx)
    x = np.zeros((N, T + 1, nx))
    u = np.zeros((N, T, nu))
    for i in range(N):
        u[i] = w[i * per:i * per + T * nu].reshape(T, nu)
        x[i, 1:] = w[i * per + T * nu:(i + 1) * per].reshape(T, nx)
        x[i, 0] = x0[i]
    return x, u


def pack_dw(ins: EqpInstance, gx, gu):
    """dL/dw from dL/dx [N][T+1][nx] and dL/du [N][T][nu] (x_0 is no variable)."""
    return np.concatenate([np.concatenate([gu[i].ravel(), gx[i, 1:].ravel()]) for i in range(ins.N)])


def implicit_gradient(ins: EqpInstance, gx, gu) -> Dict[str, np.ndarray]:
    """dL/dtheta by the implicit function theorem on the dense KKT system.

    gx [N][T+1][nx], gu [N][T][nu]: dL/dx and dL/du at the EQP solution.  The
    t = 0 entry of gx is the direct dependence of L on x_0 = x0 and is added to
    dL/dx0.  The partial derivatives of F = [H w + c + E'y ; E w - e] in
    closed form, with w_t = qT_scale at t = T and 1 before:
      log q_k:  d(H w + c)/d log q_k = 2 w_t q_k (x_t,k - r_t,k) on x_t,k, t >= 1
      log r_a:  d(H w)/d log r_a = 2 r_a u_t,a on u_t,a
      x0_i:     d(E w - e)/d x0_i = -A on the t = 0 dynamics rows of agent i
      r_i,t,k:  dc/d r_i,t,k = -2 w_t q_k on x_t,k of agent i (t >= 1)
    and dL/dtheta = -(wbar' dF_top/dtheta + ybar' dF_bot/dtheta)."""
    E, tags = constraints(ins)
    w, y = solve(ins, E=E, tags=tags)
    H, c = objective(ins)
    K = kkt_matrix(H, E)
    adj = np.linalg.solve(K, np.concatenate([pack_dw(ins, gx, gu), np.zeros(E.shape[0])]))
    wbar, ybar = adj[:H.size], adj[H.size:]
    N, T, nx, nu = ins.N, ins.T, ins.nx, ins.nu
    q, r = np.exp(ins.logq), np.exp(ins.logr)
    x, u = trajectories(ins, w)
    xb, ub = trajectories(ins, wbar)                 # the adjoint in the layout of (x, u); xb[:, 0] unused
    wt = np.ones(T + 1)
    wt[T] = ins.qT_scale
    wt[0] = 0.0                                      # x_0 is data, not a variable
    out = {}
    # log q: -sum_{i,t} wbar_x[i,t,k] * 2 w_t q_k (x - r)[i,t,k]
    out["logq"] = -np.einsum("itk,t,k,itk->k", xb, wt * 2.0, q, x - ins.xref)
    # log r: -sum_{i,t} wbar_u[i,t,a] * 2 r_a u[i,t,a]
    out["logr"] = -np.einsum("ita,a,ita->a", ub, 2.0 * r, u)
    # references: -wbar_x[i,t,k] * (-2 w_t q_k), t >= 1 (zero at t = 0)
    out["xref"] = np.einsum("itk,t,k->itk", xb, wt * 2.0, q)
    # x0: the t = 0 dynamics rows x_1 - B u_0 = A x0; dF_bot/dx0 = -A, so the
    # gradient is ybar_rows' A, plus the direct term
    g0 = np.zeros((N, nx))
    for k, tg in enumerate(tags):
        if tg[0] == "dyn" and tg[2] == 0:
            _, i, _, row = tg
            g0[i] += ybar[k] * ins.A[row]
    out["x0"] = g0 + gx[:, 0, :]
    return out


FD_STEP = dict(logq=1e-4, logr=1e-4, x0=1e-6, xref=1e-6)


def fd_gradient(ins: EqpInstance, loss, h: Optional[Dict[str, float]] = None,
                entries: Optional[Dict[str, Sequence[int]]] = None) -> Dict[str, np.ndarray]:
    """Central finite differences of loss(x, u, theta) through full EQP
    re-solves (active sets and normals fixed).  `entries` restricts a
    parameter to a subset of its flat indices (the others are left at 0).

    The KKT matrix depends on logq and logr only, so for x0 and xref one
    factorization serves every re-solve and the step is 1e-6.  The solution is
    affine in x0 and xref, so a quadratic loss makes their central difference
    exact for any step, up to rounding (about 1e-16 |L| / h).  A weight step
    re-factorizes the matrix, whose rounding (about 1e-16 cond(K) relative)
    over a 1e-6 step would leave ~1e-6 of noise; those steps are 1e-4, where
    the O(h^2) truncation is ~1e-9 relative."""
    h = dict(FD_STEP, **(h or {}))
    E, tags = constraints(ins)
    base = ins.theta()
    H0, _ = objective(ins)
    lu = sla.lu_factor(kkt_matrix(H0, E))
    out = {}
    for name in PARAMS:
        arr = base[name]
        grad = np.zeros_like(arr)
        idx = range(arr.size) if entries is None or name not in entries else entries[name]
        for k in idx:
            vals = []
            for sgn in (1.0, -1.0):
                th = {kk: vv.copy() for kk, vv in base.items()}
                th[name].reshape(-1)[k] += sgn * h[name]
                Hs, cs = objective(ins, th)
                b = np.concatenate([-cs, rhs(ins, tags, th)])
                sol = sla.lu_solve(lu, b) if name in ("x0", "xref") else np.linalg.solve(kkt_matrix(Hs, E), b)
                x, u = trajectories(ins, sol[:Hs.size], th)
                vals.append(loss(x, u, th))
            grad.reshape(-1)[k] = (vals[0] - vals[1]) / (2.0 * h[name])
        out[name] = grad
    return out


def kkt_certificate(ins: EqpInstance):
    """Is the EQP solution the minimizer of the inequality QP (Sec. III-A with
    the normals fixed)?  The QP is strictly convex, so it is iff the EQP
    solution satisfies every dropped inequality (bounds off W, half-planes off
    A_c) and every held one pushes the right way.  In the sign of F
    (H w + c + E'y = 0) the multiplier of an input at its lower bound must be
    <= 0, at its upper bound >= 0, and of a half-plane n'(p_i - p_j) >= d_min
    <= 0.  Returns (worst primal violation, worst multiplier of the wrong
    sign), both >= 0."""
    E, tags = constraints(ins)
    w, y = solve(ins, E=E, tags=tags)
    x, u = trajectories(ins, w)
    dual = 0.0
    for yk, tg in zip(y, tags):
        if tg[0] == "bound":
            lower = ins.W[tg[1], tg[2], tg[3]] == 1
            dual = max(dual, yk if lower else -yk)
        elif tg[0] == "pair":
            dual = max(dual, yk)
    free = ins.W == 0
    prim = max(0.0, float(np.max(np.where(free, ins.u_lo - u, -np.inf))),
               float(np.max(np.where(free, u - ins.u_hi, -np.inf))))
    act = set(ins.active)
    for (i, j, t), nv in ins.normals.items():
        if (i, j, t) not in act:
            prim = max(prim, ins.d_min - float(nv @ (x[i, t, :ins.nu] - x[j, t, :ins.nu])))
    return prim, dual


def kkt_condition(ins: EqpInstance) -> float:
    """Condition number of the EQP's KKT matrix (infinite when the held
    constraints are linearly dependent, where the multipliers and the x0
    gradient are not unique)."""
    E, _ = constraints(ins)
    H, _ = objective(ins)
    return float(np.linalg.cond(kkt_matrix(H, E)))
