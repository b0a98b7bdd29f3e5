"""Independent check formulation for the oracle pins.

The oracle solves each local QP over (u, x) with the dynamics as equality
rows of a dense KKT system.  The pins here instead eliminate the states
(x_t = A^t x0 + sum_s A^(t-1-s) B u_s) and write the same objective as a
linear least-squares problem ||J u - b||^2 in the inputs alone, so that a
mistake in the oracle's KKT assembly (a dropped factor of 2, a wrong sign on
the consensus term, a shifted stage index) shows up as a mismatch.
"""
from __future__ import annotations

import itertools
from typing import List, Optional, Sequence, Tuple

import numpy as np


def state_maps(A: np.ndarray, B: np.ndarray, T: int):
    """Phi[t] = A^t, Gam[t] = d x_t / d u (nx x T nu), t = 0..T."""
    nx, nu = B.shape
    Phi = [np.eye(nx)]
    for _ in range(T):
        Phi.append(A @ Phi[-1])
    Gam = [np.zeros((nx, T * nu))]
    for t in range(1, T + 1):
        G = np.zeros((nx, T * nu))
        for s in range(t):
            G[:, s * nu:(s + 1) * nu] = Phi[t - 1 - s] @ B
        Gam.append(G)
    return Phi, Gam


def agent_ls(A, B, T, x0, xref, q_diag, r_diag, qT_scale, rho=0.0, z=None, lam=None):
    """Rows of the agent objective as ||J u - b||^2.

    Objective (Eq. 1 stage costs, no 1/2):
        sum_{t=1}^{T-1} (x_t - r_t)'Q(x_t - r_t) + (x_T - r_T)'Q_T(x_T - r_T)
      + sum_{t=0}^{T-1} u_t'R u_t
      + sum_j sum_{t=1}^{T} (rho/2)||C x_t - z_j,t + lam_j,t/rho||^2
    (the t = 0 tracking term is constant).  z, lam: [n_nbr][T+1][dp].
    """
    nx, nu = B.shape
    dp = nu
    Phi, Gam = state_maps(A, B, T)
    rows, rhs = [], []
    for t in range(1, T + 1):
        w = (qT_scale if t == T else 1.0) * np.asarray(q_diag)
        s = np.sqrt(w)
        rows.append(s[:, None] * Gam[t])
        rhs.append(s * (xref[t] - Phi[t] @ x0))
    s = np.sqrt(np.asarray(r_diag))
    for t in range(T):
        R = np.zeros((nu, T * nu))
        R[:, t * nu:(t + 1) * nu] = np.diag(s)
        rows.append(R)
        rhs.append(np.zeros(nu))
    if z is not None:
        sr = np.sqrt(rho / 2.0)
        for j in range(z.shape[0]):
            for t in range(1, T + 1):
                rows.append(sr * Gam[t][:dp])
                rhs.append(sr * (z[j, t] - lam[j, t] / rho - (Phi[t] @ x0)[:dp]))
    return np.vstack(rows), np.concatenate(rhs)


def rollout(A, B, x0, u):
    T = u.shape[0]
    x = np.zeros((T + 1, A.shape[0]))
    x[0] = x0
    for t in range(T):
        x[t + 1] = A @ x[t] + B @ u[t]
    return x


def enumerate_active_sets(J, b, lo, hi, tol=1e-10):
    """Brute force over every free / lower / upper pattern of the inputs.

    For each pattern, the fixed inputs sit at their bounds and the free ones
    minimise ||J u - b||^2; a pattern is a KKT point when the free inputs are
    inside the box and the gradient 2 J'(J u - b) has the sign that a binding
    bound requires (>= 0 at a lower bound, <= 0 at an upper bound).
    Returns the list of (pattern, u) KKT points.
    """
    n = J.shape[1]
    out = []
    for pat in itertools.product((0, 1, 2), repeat=n):
        pat = np.array(pat)
        u = np.where(pat == 1, lo, np.where(pat == 2, hi, 0.0))
        free = pat == 0
        if free.any():
            Jf = J[:, free]
            sol, *_ = np.linalg.lstsq(Jf, b - J[:, ~free] @ u[~free], rcond=None)
            u[free] = sol
        if np.any(u[free] < lo[free] - tol) or np.any(u[free] > hi[free] + tol):
            continue
        g = 2.0 * J.T @ (J @ u - b)
        if np.any(np.abs(g[free]) > 1e-8 * (1 + np.abs(g).max())):
            continue
        if np.any(g[pat == 1] < -tol) or np.any(g[pat == 2] > tol):
            continue
        out.append((pat, u))
    return out
