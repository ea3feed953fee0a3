"""Parity of the HIP path with the FP64 oracle for restore with local
dynamics that are not pi-invariant (Sec. 6.2, eq. (killing-rate)): the
unadjusted random-walk jump process on the 2-D isotropic mixture, whose
killing rate k = (c_tilde u + Q^T p - p) / p needs the closed-form inflow
density Q^T p at every new state.

Tolerances as for the other kernels (test_gpu_parity): kill decisions may
differ only at near-ties, moved states within 1e-6, holding times within
1e-4; the cached log u_eff within the float32 error of its three terms;
whole-run estimates within 3 combined SE of the oracle's and of the erf
truth.
"""
import math

import numpy as np
import pytest

from tests.test_gpu_parity import _gpu_run, _pi_draws, _say, _single_step_check, _sync

from tests import chain_parity as CP

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_07148_amd import restore
    return restore


def _check_log_u_eff(R, wl, run_x, lp_g, lu_g, label):
    """The cached log u_eff of the GPU states against the oracle's at the
    same (float32) points.  u_eff = u + (q - p) / c_tilde sums three float32
    terms; each carries ~2e-5 relative error at most (log-density errors of
    the densities involved), so log u_eff is good to
    2e-5 (1 + q / c + p / c) / u_eff."""
    from oracle import oracle as O
    prob = O.Problem(wl)
    fin = np.isfinite(lp_g)
    x = run_x[fin]
    lu_o = O.log_u_eff(prob, x)
    lq = O.log_inflow(prob, x)
    lp = O.log_target(prob, x)
    ue = np.exp(lu_o)
    bound = 2e-5 * (1 + np.exp(lq) / wl.c_tilde + np.exp(lp) / wl.c_tilde) / ue
    err = np.abs(lu_g[fin] - lu_o)
    _say(f"[{label}] log u_eff: {fin.sum()} states, max err {err.max():.2e}, max err / bound "
         f"{(err / bound).max():.3f}, u_eff in [{ue.min():.3f}, {ue.max():.3g}]")
    assert np.all(err <= bound)


def test_unadjusted_single_transitions_from_pi(R):
    """From exact draws of pi (the modes, where jumps happen): kills,
    taken jumps, holding times and the new states' log p / log u_eff."""
    from workloads import gmm_iso_2d_unadjusted
    wl = gmm_iso_2d_unadjusted(n_chains=20000)
    k, a, m = _single_step_check(R, wl, x_init=_pi_draws(wl, wl.n_chains, 41), label="rwu pi")
    assert k > 1000 and m > 5000


def test_unadjusted_single_transitions_after_warmup(R):
    """After 9 steps (states everywhere, some just off the box after a
    jump): the same checks, and the cached log u_eff of every state."""
    from workloads import gmm_iso_2d_unadjusted
    wl = gmm_iso_2d_unadjusted(n_chains=20000)
    k, a, m = _single_step_check(R, wl, warm=9, label="rwu warm")
    assert k > 1000 and m > 500
    run = R.Run(R.problem_from_workload(wl))
    run.step(9)
    _sync()
    arr = run.arrays()
    x = arr["x"].cpu().numpy().T.astype(np.float64)
    lp = arr["logp"].cpu().numpy().astype(np.float64)
    lu = arr["logu"].cpu().numpy().astype(np.float64)
    run.close()
    off = ~np.isfinite(lp)
    _say(f"[rwu warm] states off the box: {off.sum()}")
    assert np.all(lu[off] == 0.0)
    _check_log_u_eff(R, wl, x, lp, lu, "rwu warm")


def test_unadjusted_whole_run_matches_oracle_and_truth(R):
    """The full 2-D workload (4096 chains x 1000 steps + drain): GPU and
    oracle estimates within 3 combined SE, both within 3 SE of the erf
    truth, every chain without a near-tie with the oracle's tour count and
    sums, no non-finite chain."""
    from oracle import oracle as O, truth
    from workloads import gmm_iso_2d_unadjusted
    wl = gmm_iso_2d_unadjusted()
    _say("[rwu run] gpu")
    est, arr = _gpu_run(R, wl)
    _say("[rwu run] oracle")
    ores = O.run(O.Problem(wl), 0, wl.n_chains)
    oest = O.estimate(ores)
    tr = truth.truths(wl)
    for key in ("p_lambda", "lam_pf", "pi_f"):
        se = math.hypot(est[key + "_se"], oest[key + "_se"])
        _say(f"[rwu run] {key}: gpu {est[key]:.6g} +- {est[key + '_se']:.2g}  oracle {oest[key]:.6g} "
             f"+- {oest[key + '_se']:.2g}  truth {tr[key]:.6g}")
        assert abs(est[key] - oest[key]) < 3 * se
        assert abs(est[key] - tr[key]) < 3 * est[key + "_se"]
    assert est["nonfinite"] == 0 and oest["nonfinite"] == 0
    assert est["tours_censored"] == 0 and oest["tours_censored"] == 0
    m = CP.check_chain_sums(arr, ores, wl, say=_say, label="rwu run")
    _say(f"[rwu run] transitions gpu {est['transitions']} oracle {oest['transitions']}; kill rate "
         f"{est['kill_rate']:.4f} accept rate {est['accept_rate']:.4f}")
    if not m["mismatch"].any():
        assert est["transitions"] == oest["transitions"]
    else:
        assert abs(est["transitions"] - oest["transitions"]) <= m["mismatch"].sum() * (wl.n_steps + wl.drain_cap)
    assert abs(est["accept_rate"] + est["kill_rate"] - 1) < 1e-9


def test_unadjusted_negative_rate_marks_the_same_chains(R):
    """c_tilde = 3.5 is just below sup (p - Q^T p) = 3.84: chains that reach
    the small region around the highest mode where the rate would be
    negative get a NaN holding time (about 40% of them within 200 steps);
    the GPU reports them as non-finite, and they are the oracle's chains
    with NaN sums (trajectories agree up to near-ties)."""
    from oracle import oracle as O
    from workloads import gmm_iso_2d_unadjusted
    wl = gmm_iso_2d_unadjusted(n_chains=4096, n_steps=200).with_(c_tilde=3.5)
    est, arr = _gpu_run(R, wl)
    ores = O.run(O.Problem(wl), 0, wl.n_chains)
    oest = O.estimate(ores)
    bad_g = ~np.isfinite(arr["t_done"])
    bad_o = ~np.isfinite(ores.t_done)
    near = CP.near_tie_chains(ores.min_margin)
    differ = bad_g != bad_o
    _say(f"[rwu negative] non-finite chains gpu {est['nonfinite']} ({bad_g.sum()}) oracle {oest['nonfinite']}; "
         f"near-tie chains {near.sum()}, chains that differ {differ.sum()} (all near-tie: {bool(np.all(near[differ]))})")
    assert 100 < est["nonfinite"] == bad_g.sum() < wl.n_chains - 100 and oest["nonfinite"] > 100
    assert not np.any(differ & ~near)


@pytest.mark.parametrize("d,K", [(1, 3), (5, 6), (16, 4)])
def test_unadjusted_single_transitions_other_shapes(R, d, K):
    """Other members of the kernel set (the smallest dimension, an odd one
    and the largest), parameters read through the scalar cache and through
    LDS (the Q^T p terms follow the components in the slab), from exact pi
    draws and after a warm-up from mu.  c_tilde = P, the sum of the
    component peaks, bounds sup p and so keeps u_eff >= 1 - p / c_tilde >= 0."""
    from workloads import gmm_iso_2d_unadjusted
    rng = np.random.default_rng(7000 + 100 * d + K)
    sig = rng.uniform(0.06, 0.12, K)
    w = rng.dirichlet(np.ones(K))
    params = {"weights": w, "means": rng.uniform(0.25, 0.75, (K, d)), "sigmas": sig}
    ct = float((w * (2 * np.pi * sig ** 2) ** (-d / 2)).sum())
    wl = gmm_iso_2d_unadjusted(n_chains=4096 + 37).with_(d=d, K=K, params=params, c_tilde=ct)
    x0 = _pi_draws(wl, wl.n_chains, 9)
    for lds in (False, True):
        _single_step_check(R, wl, x_init=x0, label=f"rwu d{d} K{K} pi lds={lds}", lds=lds)
        _single_step_check(R, wl, warm=4, label=f"rwu d{d} K{K} warm lds={lds}", lds=lds)


def test_unadjusted_rao_blackwellised_holding_time(R):
    """With RESTORE_FLAG_RB_DT the general process accumulates
    E[dt | x] = 1 / (1 + k) with its own rate k = c_tilde u_eff / p: single
    transitions after warm-up against the oracle with the same option, and
    the whole 2-D workload within 3 SE of the oracle's run and of the truth,
    with the same tours as the sampled run and no larger SE."""
    from oracle import oracle as O, truth
    from workloads import gmm_iso_2d_unadjusted
    _single_step_check(R, gmm_iso_2d_unadjusted(n_chains=8192), warm=5, label="rwu rb warm", rb=True)
    wl = gmm_iso_2d_unadjusted()
    est, _ = _gpu_run(R, wl, flags=R.FLAG_RB_DT)
    ref, _ = _gpu_run(R, wl)
    oest = O.estimate(O.run(O.Problem(wl, rb_dt=True), 0, wl.n_chains))
    tr = truth.truths(wl)
    assert est["tours_done"] == ref["tours_done"] and est["transitions"] == ref["transitions"]
    for key in ("p_lambda", "lam_pf", "pi_f"):
        _say(f"[rwu rb] {key}: gpu {est[key]:.6g} +- {est[key + '_se']:.2g} (sampled dt: +- {ref[key + '_se']:.2g}) "
             f"oracle {oest[key]:.6g} truth {tr[key]:.6g}")
        assert abs(est[key] - oest[key]) < 3 * math.hypot(est[key + "_se"], oest[key + "_se"])
        assert abs(est[key] - tr[key]) < 3 * est[key + "_se"]
        assert est[key + "_se"] <= 1.02 * ref[key + "_se"]
