"""Parity of the HIP path's MH reference chain M^l with the FP64 oracle.

M^l is the paper's baseline (Sec. 5, eq. (mixture-proposal-kernel);
Sec. 8): with c_tilde = 0 every update is a large step y ~ mu with
probability l, accepted with p(y) u(x) / (p(x) u(y)), or a small step.
Tolerances as for the restore transitions (test_gpu_parity): decisions
identical outside the near-tie margins, the large-step choice identical
everywhere (a float32-exact uniform against the float32 l on both sides),
unmoved states bit-exact, moved states within 1e-6, log p within the
float32 bound.
"""
import math

import numpy as np
import pytest

from tests import chain_parity as CP
from tests.test_gpu_parity import TAU_CAT, _c_max, _pi_draws, _say, _sync

pytestmark = pytest.mark.gpu

ELL = 0.3


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_07148_amd import restore
    return restore


def _mh_step_check(R, wl, ell, x_init, mu=None, label="", x_tol=1e-6):
    import torch
    from oracle import oracle as O
    run = R.Run(R.problem_from_workload(wl, c_tilde=0.0, mu=mu, large_step_prob=ell))
    arr = run.arrays()
    arr["x"].copy_(torch.from_numpy(np.ascontiguousarray(x_init.T.astype(np.float32))).cuda())
    run.refresh_cache()
    run.step(2)   # two steps from the loaded states, then the compared one
    _sync()
    x0 = arr["x"].cpu().numpy().T.astype(np.float64).copy()
    s = run.steps_taken
    run.step(1)
    _sync()
    x1 = arr["x"].cpu().numpy().T.astype(np.float64)
    status = arr["status"].cpu().numpy()
    lp_g = arr["logp"].cpu().numpy().astype(np.float64)
    dt_g = arr["last_dt"].cpu().numpy().astype(np.float64)
    n = wl.n_chains
    oprob = O.Problem(wl, c_tilde=0.0, mu=mu, large_step_prob=ell)
    st = O.States(x0, np.zeros(n), np.zeros(n), np.zeros_like(x0))
    new, dt_o, flags, margins = O.transitions(oprob, st, s, np.arange(n), recompute=True)
    large_g = (status & R.ST_LAST_LARGE) != 0
    large_o = (flags & O.FLAG_LARGE) != 0
    assert not np.any(status & R.ST_LAST_KILL) and not np.any(flags & O.FLAG_KILL)
    assert np.array_equal(large_g, large_o), "large-step choice differs"
    acc_g = (status & R.ST_LAST_ACCEPT) != 0
    acc_o = (flags & O.FLAG_ACCEPT) != 0
    aflip = acc_g != acc_o
    _, sa = CP.scaled_step_margins(margins)
    _say(f"[{label}] n={n} large={large_o.sum()} accepts={acc_o.sum()} (large {(acc_o & large_o).sum()}) "
         f"near-ties {(sa < CP.TAU).sum()} accept flips={aflip.sum()} "
         f"(max scaled margin {sa[aflip].max() if aflip.any() else 0:.2e})")
    assert np.all(sa[aflip] < CP.TAU), "accept decision differs outside the near-tie margin"
    same = ~aflip
    stay = same & ~acc_o
    moved = same & acc_o
    if mu is not None:
        # a learned-mu category uniform within TAU_CAT of a boundary is a near-tie
        moved &= ~(large_o & (margins[:, 2] < TAU_CAT))
    assert np.array_equal(x1[stay], x0[stay]), "rejected moves must leave x bit-identical"
    if mu is None:
        # accepted large steps with the uniform mu are the float32 uniforms
        ok = moved & large_o
        assert np.array_equal(x1[ok], new.x[ok])
    err = np.abs(x1[moved] - new.x[moved]) / np.maximum(1.0, np.abs(new.x[moved]))
    _say(f"[{label}] moved={moved.sum()} max state rel err {err.max() if moved.any() else 0:.2e}")
    assert (err.max() if moved.any() else 0.0) <= x_tol
    # the holding time of the MH chain is the Exp(1) clock t1 (float32 log)
    assert np.all(np.abs(dt_g - dt_o) <= 1e-4 * dt_o)
    fin = same & np.isfinite(new.lp)
    lerr = np.abs(lp_g[fin] - new.lp[fin])
    quad = 4e-6 * np.maximum(0.0, _c_max(wl) - new.lp[fin])
    # the two sides evaluate log p at states that differ by dx: |grad| |dx| more
    drift = np.sum(np.abs(new.g[fin]) * np.abs(x1[fin] - new.x[fin]), axis=1)
    _say(f"[{label}] max |log p| err {lerr.max() if fin.any() else 0:.2e}")
    assert np.all(lerr <= 1e-5 * np.maximum(1.0, np.abs(new.lp[fin])) + quad + drift)
    run.close()
    return large_o.sum(), (acc_o & large_o).sum()


@pytest.mark.parametrize("case", ["iso2d_rwmh", "full8d_mala", "full8d_rwmh_learned", "full8d_mala_learned",
                                  "iso2d_all_large"])
def test_mh_single_step_matches_oracle(R, case):
    from tests import helpers as H
    from workloads import gmm_full, gmm_iso_2d
    if case.startswith("iso2d"):
        wl = gmm_iso_2d(n_chains=8192)
    elif case.startswith("full8d_mala"):
        # MALA with a learned-form mu: the pairing the benchmark's MH
        # comparison with the learned mixture runs
        wl = gmm_full(n_chains=4096)
    else:
        wl = gmm_full(n_chains=4096, local="rwmh", step=0.02)
    mu = H.mixture_mu_from_target(wl) if case.endswith("learned") else None
    ell = 1.0 if case.endswith("all_large") else ELL
    _say(f"[mh step {case}] start")
    x = _pi_draws(wl, wl.n_chains, 61)
    n_large, n_large_acc = _mh_step_check(R, wl, ell, x, mu=mu, label=f"mh step {case}")
    assert n_large > 0.2 * wl.n_chains * ell
    # a uniform large step into an 8-D mode is (almost) never accepted
    assert n_large_acc > 0 or case == "full8d_mala"


@pytest.mark.parametrize("rb", [False, True])
def test_mh_whole_run_matches_oracle_and_truth(R, rb):
    """M^l on the 2-D mixture: burn-in, reset, run; the pooled ergodic
    average against the erf truth and against the oracle's run of the same
    chains, and the bookkeeping of the counters."""
    from oracle import oracle as O, truth
    from workloads import gmm_iso_2d
    wl = gmm_iso_2d(n_chains=4096)
    burn, n = 2000, 6000
    _say(f"[mh run rb={rb}] start")
    run = R.Run(R.problem_from_workload(wl, c_tilde=0.0, large_step_prob=ELL, flags=R.FLAG_RB_DT if rb else 0))
    run.step(burn)
    run.reset_sums()
    run.step(n)
    run.drain()   # nothing to finish
    est = run.estimate()
    arr = run.arrays()
    t_g = arr["t_done"].cpu().numpy()
    a_g = arr["a_done"].cpu().numpy()
    assert est["tours_done"] == 0 and est["tours_censored"] == 0 and est["kills"] == 0
    assert math.isnan(est["p_lambda"]) and math.isnan(est["lam_pf"])
    assert est["transitions"] == wl.n_chains * n
    assert abs(est["large_steps"] / est["transitions"] - ELL) < 0.005
    if rb:
        assert np.all(t_g == n)
    tr = truth.truths(wl)
    assert abs(est["pi_f"] - tr["pi_f"]) < 3 * est["pi_f_se"]
    c_or = 1024
    r = O.run(O.Problem(wl, c_tilde=0.0, large_step_prob=ELL, burn_in=burn, rb_dt=rb), 0, c_or,
              n_steps=burn + n)
    eo = O.estimate(r)
    assert eo["transitions"] == c_or * n
    # chains whose trajectories never met a near-tie agree to float32 accuracy
    n_g = arr["n_done"].cpu().numpy()
    CP.check_chain_sums({"n_done": n_g[:c_or], "t_done": t_g[:c_or], "a_done": a_g[:c_or]}, r, wl, say=_say,
                        label=f"mh run rb={rb} first {c_or} chains")
    _say(f"[mh run rb={rb}] gpu pi_f {est['pi_f']:.6g} +- {est['pi_f_se']:.2g}, oracle (first {c_or} chains) "
         f"{eo['pi_f']:.6g} +- {eo['pi_f_se']:.2g}, truth {tr['pi_f']:.6g}; large-step acceptance "
         f"{est['large_accepts'] / est['large_steps']:.3f} vs {eo['large_accepts'] / eo['large_steps']:.3f}")
    assert abs(est["pi_f"] - eo["pi_f"]) < 3 * math.hypot(est["pi_f_se"], eo["pi_f_se"])
    run.close()


def test_mh_whole_run_8d_learned_mu_matches_oracle(R):
    """M^l on the 8-D mixture with MALA small steps and large steps from a
    mixture mu of the learned form (the pairing of the benchmark's MH
    comparison with the learned mixture; 4096 chains, 2000-step burn-in, 512
    steps, unit holding times): the ergodic average within 3 SE of the Genz
    truth and of the oracle's run of the first 1024 chains, whose sums it
    reproduces chain by chain."""
    from oracle import oracle as O, truth
    from tests import helpers as H
    from workloads import gmm_full
    wl = gmm_full(n_chains=4096)
    mu = H.mixture_mu_from_target(wl)
    burn, n = 2000, 512
    _say("[mh run 8d learned mu] start")
    run = R.Run(R.problem_from_workload(wl, c_tilde=0.0, mu=mu, large_step_prob=ELL, flags=R.FLAG_RB_DT))
    run.step(burn)
    run.reset_sums()
    run.step(n)
    run.drain()
    est = run.estimate()
    arr = {k: v.cpu().numpy() for k, v in run.arrays().items() if k in ("n_done", "t_done", "a_done")}
    run.close()
    tr = truth.truths(wl)
    c_or = 1024
    r = O.run(O.Problem(wl, c_tilde=0.0, mu=mu, large_step_prob=ELL, burn_in=burn, rb_dt=True), 0, c_or,
              n_steps=burn + n)
    eo = O.estimate(r)
    CP.check_chain_sums({k: v[:c_or] for k, v in arr.items()}, r, wl, mu=mu, say=_say,
                        label=f"mh run 8d learned mu first {c_or} chains")
    _say(f"[mh run 8d learned mu] gpu pi_f {est['pi_f']:.6g} +- {est['pi_f_se']:.2g}, oracle (first {c_or}) "
         f"{eo['pi_f']:.6g} +- {eo['pi_f_se']:.2g}, truth {tr['pi_f']:.6g}; "
         f"large-step acceptance {est['large_accepts'] / est['large_steps']:.3f}")
    assert abs(est["pi_f"] - tr["pi_f"]) < 3 * est["pi_f_se"]
    assert abs(est["pi_f"] - eo["pi_f"]) < 3 * math.hypot(est["pi_f_se"], eo["pi_f_se"])


def test_reset_sums_only_for_the_mh_chain(R):
    from workloads import gmm_iso_2d
    wl = gmm_iso_2d(n_chains=1024)
    run = R.Run(R.problem_from_workload(wl))
    with pytest.raises(R.RestoreError) as e:
        run.reset_sums()
    assert e.value.status == R.E_BAD_STATE
    run.close()
    run = R.Run(R.problem_from_workload(wl, c_tilde=0.0, large_step_prob=ELL))
    run.step(50)
    run.reset_sums()
    est = run.estimate()
    assert est["transitions"] == 0 and est["large_steps"] == 0
    arr = run.arrays()
    assert float(arr["t_done"].abs().sum()) == 0.0 and float(arr["a_done"].abs().sum()) == 0.0
    x_before = arr["x"].clone()
    run.step(1)
    assert run.estimate()["transitions"] == 1024
    assert run.steps_taken == 51 and not bool((arr["x"] == x_before).all())
    run.drain()
    with pytest.raises(R.RestoreError):
        run.reset_sums()
    run.close()


def test_mh_image_splats_cover_the_chain_time(R):
    """The MH chain on the rendering-shaped integrand splats dt at every
    pre-transition pixel: the image total equals the total chain time."""
    from workloads import pss_render
    wl = pss_render(n_chains=16384, image=(128, 128), image_batches=1)
    run = R.Run(R.problem_from_workload(wl, c_tilde=0.0, large_step_prob=ELL))
    run.step(40)
    run.reset_sums()
    run.step(60)
    _sync()
    tot = float(run.arrays()["t_done"].sum())
    img = float(run.image.double().sum())
    _say(f"[mh image] image total {img:.6g} chain time {tot:.6g}")
    assert abs(img - tot) <= 1e-4 * tot
    run.close()


def test_theorem_b_ordering_at_scale(R):
    """Theorem B of the supplement on the GPU: with c_tilde >= l / 2 the
    restore process has a time-average variance constant of f = p no larger
    than the continuous-time MH chain M^l (Exp(1) holding times), here with
    the paper's burn-in of 10,000 iterations and 2^16 chains per method."""
    from workloads import gmm_iso_2d
    C = 1 << 16
    wl = gmm_iso_2d(n_chains=C)

    def sigma2(run):
        arr = run.arrays()
        A = arr["a_done"].cpu().numpy()
        T = arr["t_done"].cpu().numpy()
        R_ = A.sum() / T.sum()
        e = (A - R_ * T) ** 2
        s2 = e.sum() / T.sum()
        se = math.sqrt(((e - s2 * T) ** 2).sum() / ((C - 1) * C)) / T.mean()
        return s2, se

    mh = R.Run(R.problem_from_workload(wl, c_tilde=0.0, large_step_prob=ELL))
    mh.step(10000)
    mh.reset_sums()
    mh.step(10000)
    s_mh, se_mh = sigma2(mh)
    mh.close()
    res = {}
    for ct in (ELL / 2, 1.0):
        rs = R.Run(R.problem_from_workload(wl, c_tilde=ct))
        rs.step(2000)
        rs.drain()
        assert rs.estimate()["tours_censored"] == 0
        res[ct] = sigma2(rs)
        rs.close()
    _say(f"[theorem B] sigma^2 MH {s_mh:.4g} +- {se_mh:.2g}; restore " +
         ", ".join(f"c~={ct:g}: {s:.4g} +- {se:.2g}" for ct, (s, se) in res.items()))
    for ct, (s, se) in res.items():
        assert s < s_mh + 3 * math.hypot(se, se_mh), ct
    assert res[1.0][0] < 0.6 * s_mh
