"""The oracle pins must catch plausible mistakes.

Each case plants one mistake in a copy of the C oracle (a dropped factor, a
flipped sign, a shifted index, a transposed operand), builds it into a
temporary library on the CPU, and runs the pin functions of
test_oracle_pins.py against it: at least one pin has to fail.  The committed
oracle itself is never modified.
"""
import ctypes
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "tadmm_oracle.c")

MUTANTS = {
    "hessian_factor_2_dropped": ("q->Hd[k] = 2.0 * wq +", "q->Hd[k] = 1.0 * wq +"),
    "consensus_term_sign": ("- (r < q->dp && ysum ? ysum[t * q->dp + r] : 0.0);",
                            "+ (r < q->dp && ysum ? ysum[t * q->dp + r] : 0.0);"),
    "terminal_weight_index": ("(t == T ? prm->qT_scale : 1.0)", "(t == T - 1 ? prm->qT_scale : 1.0)"),
    "projection_half_step": ("a[c] += 0.5 * v * n[c]; b[c] -= 0.5 * v * n[c];",
                             "a[c] += v * n[c]; b[c] -= v * n[c];"),
    "dual_update_sign": ("lam[ZI(i, j, t) + c] += rho * (xi[c] - a[c]);",
                         "lam[ZI(i, j, t) + c] -= rho * (xi[c] - a[c]);"),
    "multiplier_sign": ("m = (W[k] == 1) ? -y : y;", "m = (W[k] == 1) ? y : -y;"),
    "normal_orientation": ("n[c] = (pi[c] - pj[c]) / dd;", "n[c] = (pj[c] - pi[c]) / dd;"),
    "dynamics_A_transposed": ("const double a = q->A[r * nx + c];", "const double a = q->A[c * nx + r];"),
    "dual_residual_no_previous": ("rho * (zs[c] - zsum_old[((size_t)i * T + (t - 1)) * dp + c]);", "rho * zs[c];"),
    "primal_residual_term": ("r2 += (pi[c] - zc) * (pi[c] - zc);", "r2 += zc * zc;"),
    "consensus_init_zero": ("z[ZI(i, j, t) + k] = sc->xref[((size_t)i * (T + 1) + t) * nx + k];",
                            "z[ZI(i, j, t) + k] = 0.0;"),
    "never_drops_negative_multiplier": ("if (drop >= 0 && mu_min < -prm->mu_tol) {", "if (0) {"),
    "adaptive_rho_keeps_stale_hessian": ("for (int i = 0; i < N; ++i) qp_ws_set_rho(&qs[i], rho);", "(void)qs;"),
    "agent_weights_of_the_first_agent": ("return sc->agent_q ? sc->agent_q + (size_t)i * nx : sc->q_diag;",
                                         "return sc->agent_q ? sc->agent_q : sc->q_diag;"),
    "agent_box_ignored": ("if (sc->agent_lo) qs[i].lo = sc->agent_lo + (size_t)i * nu;", ""),
    "state_box_dual_not_updated": ("mb[o] += sigma * (xv - yn);", "(void)0;"),
    "state_box_missing_hessian_term": ("(state_boxed(prm, r) ? prm->rho : 0.0)", "0.0"),
    "position_box_bounds_of_the_velocities": ("return r < prm->dp ? prm->p_hi[r] : prm->s_hi[r - prm->dp];",
                                              "return prm->s_hi[r % prm->dp];"),
    "adaptive_rho_drops_box_hessian_term": ("+ (state_boxed(q->prm, r) ? q->prm->rho : 0.0);", ";"),
    "agent_dynamics_of_the_first_agent": ("if (sc->agent_A) qs[i].A = sc->agent_A + (size_t)i * nx * nx;",
                                          "if (sc->agent_A) qs[i].A = sc->agent_A;"),
    "agent_input_matrix_ignored_in_kkt": ("const double b = q->B[r * nu + c];", "const double b = prm->B[r * nu + c];"),
    "momentum_weight_without_minus_one": ("const double beta = (mom_a - 1.0) / an;", "const double beta = mom_a / an;"),
    "momentum_restart_to_the_current_iterate": ("memcpy(zh, zp, zsz * sizeof(double));",
                                                "memcpy(zh, z, zsz * sizeof(double));"),
    "relaxation_dual_update_unrelaxed": ("lam[ZI(i, j, t) + c] += rho * (xi[c] - a[c]);",
                                         "lam[ZI(i, j, t) + c] += rho * (pi[c] - a[c]);"),
    "fallback_normal_rot90_sign": ("if (dp == 2) { c[0] = -v[1]; c[1] = v[0]; }",
                                   "if (dp == 2) { c[0] = v[1]; c[1] = -v[0]; }"),
    "fallback_normal_cross_axis_of_the_largest_component": (
        "for (int k = 1; k < 3; ++k) if (fabs(v[k]) < fabs(v[kmin])) kmin = k;",
        "for (int k = 1; k < 3; ++k) if (fabs(v[k]) > fabs(v[kmin])) kmin = k;"),
    "fallback_normal_ties_to_the_highest_axis": (
        "for (int k = 1; k < 3; ++k) if (fabs(v[k]) < fabs(v[kmin])) kmin = k;",
        "for (int k = 1; k < 3; ++k) if (fabs(v[k]) <= fabs(v[kmin])) kmin = k;"),
    "fallback_normal_e2_without_relative_motion": ("n[k] = (k == 0) ? 1.0 : 0.0;", "n[k] = (k == 1) ? 1.0 : 0.0;"),
    "relaxation_weights_swapped": ("prm->alpha * pi[c] + (1.0 - prm->alpha) * z[ZI(i, j, t) + c]",
                                   "(1.0 - prm->alpha) * pi[c] + prm->alpha * z[ZI(i, j, t) + c]"),
}

# The fast pins (each well under a second on the committed oracle).  Mistakes
# that the active-set method corrects by itself on the way to the unique
# optimum (a wrong side recorded for a clipped start, a wrong bound in the
# ratio test) leave every output unchanged and are not listed above.
PIN_FUNCS = [pins.test_agent_qp_unconstrained_matches_condensed_least_squares,
             pins.test_agent_qp_long_horizon_first_gain_is_dare,
             pins.test_agent_qp_bounded_matches_bvls,
             pins.test_agent_qp_tiny_horizon_brute_force,
             pins.test_agent_qp_dynamics_and_box_feasible,
             pins.test_admm_point_symmetry,
             pins.test_admm_duals_antisymmetric_and_along_normal,
             pins.test_admm_consensus_copies_satisfy_half_planes,
             pins.test_admm_residual_history_consistent_with_iterates,
             pins.test_admm_translation_invariance,
             pins.test_admm_single_agent_converges_first_iteration,
             pins.test_admm_frozen_limit_is_centralized_qp_kkt_certificate,
             pins.test_admm_adaptive_rho_frozen_limit_is_the_same_kkt_point,
             pins.test_hetero_single_agent_is_its_local_qp,
             pins.test_hetero_agent_permutation_equivariance,
             pins.test_admm_state_box_frozen_limit_is_centralized_qp_kkt_certificate,
             pins.test_admm_position_box_frozen_limit_is_centralized_qp_kkt_certificate,
             pins.test_admm_position_box_with_adaptive_rho_same_certified_limit,
             pins.test_agent_dynamics_satisfied_per_agent,
             pins.test_agent_dynamics_single_agent_is_its_local_qp,
             pins.test_agent_input_gain_is_a_reparametrization,
             pins.test_admm_relaxation_closed_form_far_apart,
             pins.test_admm_momentum_closed_form_far_apart,
             pins.test_admm_momentum_frozen_limit_is_the_same_kkt_point,
             pins.test_admm_relaxation_frozen_limit_is_the_same_kkt_point,
             pins.test_fallback_normal_2d_turns_the_relative_velocity_counterclockwise,
             pins.test_fallback_normal_3d_crosses_the_smallest_velocity_axis,
             pins.test_fallback_normal_3d_ties_go_to_the_lowest_axis,
             pins.test_fallback_normal_is_e1_without_relative_motion,
             pins.test_fallback_normal_reference_position_first,
             pins.test_frozen_reference_normals_of_an_exact_swap_use_the_velocity_rule]


def _call_pin(fn):
    """Run one pin with default parametrisation; returns True if it passed."""
    import inspect
    params = inspect.signature(fn).parameters
    kw = {}
    for name in params:
        if name == "dp":
            kw[name] = 2
        elif name == "seed":
            kw[name] = 0
        elif name == "T":
            kw[name] = 3
        elif name == "start":
            kw[name] = oracle.START_COLD
        elif name == "alpha":
            kw[name] = 1.5
    try:
        fn(**kw)
        return True
    except (AssertionError, RuntimeError, ValueError, FloatingPointError, ZeroDivisionError, IndexError):
        return False


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mut = tmp_path / "oracle_mut.c"
    mut.write_text(src.replace(old, new))
    hdr = os.path.join(os.path.dirname(SRC), "tadmm_oracle.h")
    (tmp_path / "tadmm_oracle.h").write_text(open(hdr).read())
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", str(mut), "-o", str(so), "-lm"],
                   check=True, capture_output=True)
    saved = oracle._lib
    try:
        oracle._lib = None
        orig_build = oracle.build
        oracle.build = lambda force=False: str(so)
        try:
            oracle.lib()
            results = {fn.__name__: _call_pin(fn) for fn in PIN_FUNCS}
        finally:
            oracle.build = orig_build
    finally:
        oracle._lib = saved
    failed = [k for k, ok in results.items() if not ok]
    assert failed, f"no pin caught mutant {name}"
