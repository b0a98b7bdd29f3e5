"""Pins of the oracle's gradient through a converged solve (oracle/grad.py).

The equality QP is pinned to the C oracle's converged ADMM solution (a
different formulation and code), its implicit gradient to central finite
differences of full re-solves, and both to closed forms in the special cases
where the gradient has one: the unconstrained LQR (states eliminated, an affine
map of x0 and the references), and a fully saturated agent (the states are a
pure function of x0)."""
import functools

import numpy as np
import pytest

import oracle
import synth
from oracle import grad as G
from tests import condensed
from tests import grad_common as GC


@functools.lru_cache(maxsize=1)
def _cases():
    ids = [5, 7]
    p, scs = synth.config3(S=len(ids), scenario_ids=ids)
    cases = GC.build_cases(p, scs, ids, want=2, threads=0)
    assert [c.sid for c in cases] == ids
    return p, cases


def _pref(ins):
    return ins.xref[:, :, :ins.nu].copy()


def _loss(pref):
    return lambda x, u, th: float(np.sum((x[:, :, :pref.shape[2]] - pref) ** 2))


def _check_eqp_is_admm_solution(c):
    w, _ = G.solve(c.ins)
    x, u = G.trajectories(c.ins, w)
    # the ADMM stopped at eps 1e-8 on its (Boyd) residuals, which leaves up to
    # a few 1e-5 on single inputs (R is small)
    rel = GC.rel_err(np.concatenate([x.ravel(), u.ravel()]), np.concatenate([c.res["x"].ravel(), c.res["u"].ravel()]))
    assert rel < 1e-5 and np.abs(u - c.res["u"]).max() < 1e-4, rel


def test_eqp_solution_is_the_converged_admm_solution():
    """Sec. III-A: with the normals frozen the ADMM limit is the QP minimizer,
    which the EQP on the final active sets reproduces."""
    _, cases = _cases()
    for c in cases:
        _check_eqp_is_admm_solution(c)
        assert c.cert[0] <= GC.CERT_TOL and c.cert[1] <= GC.CERT_TOL


def _losses(ins, x, u):
    """The tracking loss of the differentiation workload, and a random linear
    loss (which also reaches u and the t = 0 state)."""
    pref = _pref(ins)
    _, gx, gu = GC.tracking_loss_grads(ins, x, u, pref)
    rng = np.random.default_rng(4)
    ax, au = rng.normal(size=x.shape), rng.normal(size=u.shape)
    return [(gx, gu, _loss(pref)), (ax, au, lambda x, u, th: float(np.sum(ax * x) + np.sum(au * u)))]


def _check_implicit_vs_fd(ins, grad_fn=G.implicit_gradient):
    w, _ = G.solve(ins)
    x, u = G.trajectories(ins, w)
    rng = np.random.default_rng(0)
    ent = dict(x0=rng.choice(ins.x0.size, 12, replace=False), xref=rng.choice(ins.xref.size, 40, replace=False))
    ent["xref"] = np.concatenate([ent["xref"], [ins.xref[0].size * 2 + 4 * ins.T + 1]])   # a terminal entry
    for gx, gu, loss in _losses(ins, x, u):
        g = grad_fn(ins, gx, gu)
        fd = G.fd_gradient(ins, loss, h=dict(x0=1e-4, xref=1e-4), entries=ent)
        for name in G.PARAMS:
            idx = np.arange(g[name].size) if name not in ent else np.asarray(ent[name])
            a, b = g[name].reshape(-1)[idx], fd[name].reshape(-1)[idx]
            scale = max(np.abs(g[name]).max(), 1e-12)
            assert np.abs(a - b).max() <= 1e-7 * scale, (name, np.abs(a - b).max() / scale)
        # the references reach the solution only at t >= 1
        assert np.all(g["xref"][:, 0, :] == 0.0)


def test_implicit_gradient_matches_central_differences_of_resolves():
    """Implicit function theorem vs central FD (FP64) of the frozen EQP, step
    1e-4: the loss is quadratic in x0 and the references (the solution is
    affine in them), where any step is exact and 1e-4 keeps the rounding of a
    loss of a few hundred below 1e-9 relative; on the log-weights the O(h^2)
    truncation is ~1e-9."""
    _, cases = _cases()
    _check_implicit_vs_fd(cases[1].ins)


def _free_instance(N=2, T=8, W=None, seed=3):
    p = synth.ProblemParams(dp=2, u_max=2.0)
    rng = np.random.default_rng(seed)
    x0 = np.zeros((N, p.nx))
    x0[:, :2] = rng.uniform(-3, 3, (N, 2))
    x0[:, 2:] = rng.normal(0, 0.3, (N, 2))
    goals = rng.uniform(-3, 3, (N, 2))
    xref = synth.straight_line_ref(x0[:, :2], goals, T)
    xref = xref + rng.normal(0, 0.1, xref.shape)
    ins = G.EqpInstance(A=p.A, B=p.B, u_lo=p.u_lo, u_hi=p.u_hi, qT_scale=p.qT_scale, d_min=p.d_min,
                        x0=x0, xref=xref, logq=np.log(p.q_diag) + rng.normal(0, 0.2, p.nx),
                        logr=np.log(p.r_diag) + rng.normal(0, 0.2, p.nu),
                        W=np.zeros((N, T, p.nu), np.int64) if W is None else W, active=[], normals={})
    return p, ins


def _condensed_solution(ins, i, x0, xref, logq, logr):
    J, b = condensed.agent_ls(ins.A, ins.B, ins.T, x0, xref, np.exp(logq), np.exp(logr), ins.qT_scale)
    u = np.linalg.lstsq(J, b, rcond=None)[0].reshape(ins.T, ins.nu)
    return condensed.rollout(ins.A, ins.B, x0, u), u


def test_unconstrained_gradient_matches_condensed_lqr():
    """No bound and no half-plane held: each agent is a finite-horizon LQR.
    In the condensed form (states eliminated) the solution is an affine map of
    x0 and of the references, so unit perturbations give its exact Jacobian;
    the weights are checked by differences of the condensed solve."""
    _, ins = _free_instance()
    rng = np.random.default_rng(1)
    gx = rng.normal(size=(ins.N, ins.T + 1, ins.nx))
    gu = rng.normal(size=(ins.N, ins.T, ins.nu))
    g = G.implicit_gradient(ins, gx, gu)
    for i in range(ins.N):
        L = lambda x, u: float(np.sum(gx[i] * x) + np.sum(gu[i] * u))
        base = L(*_condensed_solution(ins, i, ins.x0[i], ins.xref[i], ins.logq, ins.logr))
        for k in range(ins.nx):
            e = np.zeros(ins.nx)
            e[k] = 1.0
            d = L(*_condensed_solution(ins, i, ins.x0[i] + e, ins.xref[i], ins.logq, ins.logr)) - base
            assert d == pytest.approx(g["x0"][i, k], rel=1e-8, abs=1e-8)
        for t in (0, 1, ins.T // 2, ins.T):
            for k in range(ins.nx):
                xr = ins.xref[i].copy()
                xr[t, k] += 1.0
                d = L(*_condensed_solution(ins, i, ins.x0[i], xr, ins.logq, ins.logr)) - base
                assert d == pytest.approx(g["xref"][i, t, k], rel=1e-8, abs=1e-8)
    h = 1e-5
    for name, size in (("logq", ins.nx), ("logr", ins.nu)):
        for k in range(size):
            tot = 0.0
            for i in range(ins.N):
                L = lambda x, u: float(np.sum(gx[i] * x) + np.sum(gu[i] * u))
                vals = []
                for s in (1.0, -1.0):
                    lq, lr = ins.logq.copy(), ins.logr.copy()
                    (lq if name == "logq" else lr)[k] += s * h
                    vals.append(L(*_condensed_solution(ins, i, ins.x0[i], ins.xref[i], lq, lr)))
                tot += (vals[0] - vals[1]) / (2 * h)
            assert tot == pytest.approx(g[name][k], rel=1e-6, abs=1e-9)


def test_saturated_agents_gradient_is_the_state_transition():
    """Every input held at a bound and no half-plane: the states are
    x_t = A^t x0 + (bound terms), so dL/dx0 = sum_t (A^t)' dL/dx_t and the
    weights and references have no influence."""
    N, T = 2, 6
    W = np.where(np.arange(T * 2).reshape(1, T, 2) % 3 == 0, 2, 1).repeat(N, 0)
    _, ins = _free_instance(N=N, T=T, W=W)
    rng = np.random.default_rng(2)
    gx = rng.normal(size=(N, T + 1, ins.nx))
    gu = rng.normal(size=(N, T, ins.nu))
    g = G.implicit_gradient(ins, gx, gu)
    Phi, _ = condensed.state_maps(ins.A, ins.B, T)
    for i in range(N):
        want = sum(Phi[t].T @ gx[i, t] for t in range(T + 1))
        np.testing.assert_allclose(g["x0"][i], want, rtol=1e-8, atol=1e-8)
    assert np.abs(g["logq"]).max() < 1e-8 and np.abs(g["logr"]).max() < 1e-8
    assert np.abs(g["xref"]).max() < 1e-8


def test_certificate_rejects_wrong_active_sets():
    """Dropping a binding half-plane lets the solution cross it; holding a
    slack one needs a multiplier of the wrong sign."""
    _, cases = _cases()
    ins = cases[1].ins
    drop = G.EqpInstance(**{**ins.__dict__, "active": ins.active[1:]})
    assert G.kkt_certificate(drop)[0] > 1e-4
    w, _ = G.solve(ins)
    x, _ = G.trajectories(ins, w)
    held = set(ins.active)
    gap = {k: float(ins.normals[k] @ (x[k[0], k[2], :2] - x[k[1], k[2], :2])) - ins.d_min
           for k in ins.normals if k not in held}
    slack = min((k for k in gap if gap[k] > 0.05), key=gap.get)
    add = G.EqpInstance(**{**ins.__dict__, "active": ins.active + [slack]})
    assert G.kkt_certificate(add)[1] > 1e-6


# ---------------------------------------------------------------------------
# planted mistakes: each must make one of the pins above fail
# ---------------------------------------------------------------------------

def _objective_no_terminal_weight(ins, theta=None):
    H, c = _ORIG["objective"](ins, theta)
    n, iu, ix = G._layout(ins)
    for i in range(ins.N):
        s = ix(i, ins.T, 0)
        H[s:s + ins.nx] /= ins.qT_scale
        c[s:s + ins.nx] /= ins.qT_scale
    return H, c


def _objective_no_factor_two(ins, theta=None):
    H, c = _ORIG["objective"](ins, theta)
    return H / 2.0, c


def _constraints_wrong_partner_sign(ins):
    E, tags = _ORIG["constraints"](ins)
    n, iu, ix = G._layout(ins)
    for k, tg in enumerate(tags):
        if tg[0] == "pair":
            _, i, j, t = tg
            E[k, ix(j, t, 0):ix(j, t, 0) + ins.nu] *= -1.0
    return E, tags


def _rhs_transposed_dynamics(ins, tags, theta=None):
    e = _ORIG["rhs"](ins, tags, theta)
    x0 = ins.x0 if theta is None else theta["x0"]
    for k, tg in enumerate(tags):
        if tg[0] == "dyn" and tg[2] == 0:
            e[k] = float(ins.A[:, tg[3]] @ x0[tg[1]])
    return e


_ORIG = dict(objective=G.objective, constraints=G.constraints, rhs=G.rhs)


@pytest.mark.parametrize("name,fn", [("objective", _objective_no_terminal_weight),
                                     ("objective", _objective_no_factor_two),
                                     ("constraints", _constraints_wrong_partner_sign),
                                     ("rhs", _rhs_transposed_dynamics)])
def test_mutant_equality_qp_is_caught(monkeypatch, name, fn):
    _, cases = _cases()
    monkeypatch.setattr(G, name, fn)
    with pytest.raises(AssertionError):
        for c in cases:
            _check_eqp_is_admm_solution(c)


@pytest.mark.parametrize("mutant", ["sign", "no_direct_x0", "no_state_multiplier"])
def test_mutant_implicit_gradient_is_caught(monkeypatch, mutant):
    _, cases = _cases()
    ins = cases[1].ins

    def bad(ins, gx, gu):
        g = G.implicit_gradient(ins, gx, gu)
        if mutant == "sign":
            return {k: -v for k, v in g.items()}
        if mutant == "no_direct_x0":
            g["x0"] = g["x0"] - gx[:, 0, :]
            return g
        # dropping the dynamics-row multiplier leaves x0 with its direct term only
        g["x0"] = gx[:, 0, :].copy()
        return g

    with pytest.raises(AssertionError):
        _check_implicit_vs_fd(ins, grad_fn=bad)
