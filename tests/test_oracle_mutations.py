"""The pins are sensitive: each plausible mistake planted in a copy of the
oracle's C source (a wrong sign, a dropped factor, a swapped operand, a
wrong index) makes at least one pin fail.  Everything here runs on the CPU
and never touches the HIP path."""
import os
import subprocess

import pytest

from oracle import oracle as O
from tests import test_oracle_general as gen
from tests import test_oracle_hmc as hmc
from tests import test_oracle_mh as mh
from tests import test_oracle_pins as pins
from tests import test_oracle_tiles as tiles

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "restore_oracle.c")

MUTATIONS = {
    # killing rate k = c u / p inverted to c p / u
    "kill_rate_inverted": ("log_k = log(cfg->c_tilde) + st->lu - st->lp;",
                           "log_k = log(cfg->c_tilde) + st->lp - st->lu;",
                           [lambda: pins.test_jump_chain_leaves_nu_invariant(None, "rwmh", 0.05, 1.0)]),
    # holding time drawn with rate 2 instead of 1
    "holding_rate_two": ("double t1 = -log(head[0]);", "double t1 = -0.5 * log(head[0]);",
                         [lambda: pins.test_kill_and_clock_law_at_fixed_state(None, "mode")]),
    # tie goes to the local move instead of the kill
    "kill_uses_t2_only": ("if (t1 < t2) {", "if (t1 < 2.0 * t2) {",
                          [lambda: pins.test_kill_and_clock_law_at_fixed_state(None, "mode")]),
    # Langevin drift with the wrong sign in the proposal
    "mala_drift_sign": ("if (lk->kind == OR_LOCAL_MALA) y[i] += 0.5",
                        "if (lk->kind == OR_LOCAL_MALA) y[i] -= 0.5",
                        [lambda: pins.test_local_kernel_alone_is_pi_invariant(None, "mala", 0.03)]),
    # reverse proposal density evaluated with the forward gradient
    "mala_reverse_uses_forward_grad": ("log_q(lk, d, y, gy, st->x)", "log_q(lk, d, y, st->g, st->x)",
                                       [lambda: pins.test_local_kernel_alone_is_pi_invariant(None, "mala", 0.03)]),
    # Box-Muller radius missing its factor 2
    "box_muller_radius": ("double r = sqrt(-2.0 * log(cand[2 * m]));", "double r = sqrt(-log(cand[2 * m]));",
                          [lambda: pins.test_normals_and_exponentials_from_steps(None)]),
    # Philox multiplier constants swapped between the two lanes
    "philox_swapped_multipliers": ("uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;",
                                   "uint64_t p0 = (uint64_t)M1 * (uint64_t)c0;",
                                   [lambda: pins.test_philox_known_answers(None)]),
    # integrand evaluated at the post-transition state instead of x_{i-1}
    "integrand_after_move": ("double f = lp_prev == -INFINITY ? 0.0 : exp(lp_prev);",
                             "double f = st.lp == -INFINITY ? 0.0 : exp(st.lp);",
                             [lambda: pins.test_whole_run_2d_matches_erf_closed_form(None)]),
    # Mahalanobis form with the mean subtracted on one side only
    "quadratic_form_index": ("q += (x[i] - m[i]) * P[i * d + j] * (x[j] - m[j]);",
                             "q += (x[i] - m[i]) * P[i * d + j] * (x[j] - m[i]);",
                             [lambda: pins.test_log_target_matches_scipy(None, pins.gmm_full)]),
    # gradient of the mixture without the responsibilities
    "grad_no_responsibility": ("double r = exp(a[k] - lp);", "double r = 1.0 / t->K;",
                               [lambda: pins.test_grad_log_target_central_differences(None, pins.gmm_iso_2d)]),
    # mu density missing the defensive uniform share
    "mu_density_drops_defensive": ("a[mu->K] = in_box(d, y) ? log(mu->beta) : -INFINITY;",
                                   "a[mu->K] = -INFINITY;",
                                   [lambda: pins.test_whole_run_8d_mixture_mu_matches_genz_truth(None)]),
    # conditional-mean holding time 1/k instead of 1/(1 + k)
    "rb_holding_time_without_holding_rate": ("return 1.0 / (1.0 + exp(log_k));", "return exp(-log_k);",
                                             [lambda: pins.test_zero_step_rao_blackwellised_moments(None)]),
    # large step accepted with the target ratio alone (u(x) / u(y) dropped)
    "large_step_drops_mu_ratio": ("lratio = (lpy + st->lu) - (st->lp + luy);", "lratio = lpy - st->lp;",
                                  [lambda: mh.test_large_step_with_proposal_equal_to_target_always_accepted(None)]),
    # independence ratio with u(y) / u(x) in place of u(x) / u(y)
    "large_step_mu_ratio_inverted": ("lratio = (lpy + st->lu) - (st->lp + luy);",
                                     "lratio = (lpy + luy) - (st->lp + st->lu);",
                                     [lambda: mh.test_large_step_with_proposal_equal_to_target_always_accepted(None),
                                      lambda: mh.test_mixture_kernel_is_pi_invariant(None, "rwmh", 0.05, "mismatched")]),
    # large step taken with probability 1 - l
    "large_step_share_complement": ("large = ul[0] < lk->large_step_prob;", "large = ul[0] >= lk->large_step_prob;",
                                    [lambda: mh.test_large_step_share_is_l(None)]),
    # the MH chain's burn-in steps accumulated
    "mh_burn_in_ignored": ("int counted = !mh || s >= cfg->burn_in;", "int counted = 1;",
                           [lambda: mh.test_mh_ergodic_average_matches_erf_truth(None, True)]),
    # HMC kinetic energy difference with the wrong sign
    "hmc_kinetic_sign": ("kinetic += 0.5 * (z[i] * z[i] - rho[i] * rho[i]);",
                         "kinetic += 0.5 * (rho[i] * rho[i] - z[i] * z[i]);",
                         [lambda: hmc.test_one_leapfrog_step_is_mala(None),
                          lambda: hmc.test_hmc_is_pi_invariant(None)]),
    # leapfrog without the closing half momentum step
    "leapfrog_full_last_kick": ("double h = (l == n - 1) ? 0.5 * e : e;", "double h = e;",
                                [lambda: hmc.test_leapfrog_is_reversible_and_volume_preserving(None)]),
    # leapfrog opening half step against the gradient
    "leapfrog_first_kick_sign": ("for (int i = 0; i < d; ++i) rho[i] += 0.5 * e * g[i];",
                                 "for (int i = 0; i < d; ++i) rho[i] -= 0.5 * e * g[i];",
                                 [lambda: hmc.test_one_leapfrog_step_is_mala(None)]),
    # tile-stratified chains not restricted to their tile
    "tile_region_dropped": ("if (cfg && chain_tile(cfg, chain, r)) {", "if (0 && chain_tile(cfg, chain, r)) {",
                            [lambda: tiles.test_chains_stay_in_their_tile(None)]),
    # tile-uniform mu drawn from the wrong corner
    "tile_sample_offset": ("(float)cand[0], (float)r[0])", "(float)cand[0], (float)r[1])",
                           [lambda: tiles.test_initial_states_lie_in_their_tiles(None)]),
    # chains dealt to tiles round-robin instead of in contiguous ranges
    "tile_map_round_robin": ("int64_t t = (int64_t)chain * T / cfg->n_chains_total;",
                             "int64_t t = (int64_t)chain % T;",
                             [lambda: tiles.test_chains_stay_in_their_tile(None)]),
    # inflow density of the unadjusted jump process without the jump variance
    "inflow_variance_without_jump": ("ak += -0.5 * log(2.0 * M_PI * (v + s)) - 0.5 * dx * dx / (v + s)",
                                     "ak += -0.5 * log(2.0 * M_PI * v) - 0.5 * dx * dx / (v + s)",
                                     [lambda: gen.test_inflow_matches_quadrature(None)]),
    # truncation factor centred with the weights of x and m swapped
    "inflow_center_swapped": ("double c = (m[i] * s + x[i] * v) / (v + s);",
                              "double c = (x[i] * s + m[i] * v) / (v + s);",
                              [lambda: gen.test_inflow_matches_quadrature(None)]),
    # general killing rate without the outflow term -p of L* p
    "general_rate_drops_outflow": ("double ue = u + (q - p) / c_tilde;", "double ue = u + q / c_tilde;",
                                   [lambda: gen.test_kill_law_uses_the_general_rate(None, "mode")]),
    # the unadjusted jump put through a Metropolis-Hastings test
    "unadjusted_jump_gets_mh_test": ("if (st->lp == -INFINITY || (!large && lk->kind == OR_LOCAL_RW_UNADJUSTED)) {",
                                     "if (st->lp == -INFINITY) {",
                                     [lambda: gen.test_kill_law_uses_the_general_rate(None, "tail")]),
    # a negative killing rate silently clamped to zero
    "negative_rate_clamped": ("return ue >= 0.0 ? log(ue) : NAN;", "return log(fmax(ue, 0.0));",
                              [lambda: gen.test_negative_rate_marks_the_chain(None)]),
    # a completed tour not counted
    "tour_not_counted": ("a_done += a_cur; t_done += t_cur; ++n_done;",
                         "a_done += a_cur; t_done += t_cur;",
                         [lambda: pins.test_whole_run_2d_matches_erf_closed_form(None)]),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path, oracle_lib):
    old, new, checks = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-o", str(lib),
                    str(mutated), "-lm", "-lpthread"], check=True)
    caught = False
    with O.use_library(str(lib)):
        for check in checks:
            try:
                check()
            except AssertionError:
                caught = True
    assert caught, f"no pin caught the planted mistake {name}"
