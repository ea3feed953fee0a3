"""Pins of the oracle's Metropolis-Hastings reference chain M^l -- no GPU.

M^l (Sec. 5, eq. (mixture-proposal-kernel); Sec. 8) is the MH chain whose
proposal is the large-step distribution mu with probability l and the small
step kernel otherwise, taken as the mixture of two MH kernels
K_l = l K_1 + (1 - l) K_0 (Theorem B of the supplement).  With c_tilde = 0
the oracle runs it; these checks pin it to facts that do not come from the
oracle itself:

* every mixture of pi-invariant MH kernels leaves pi invariant: exact pi
  draws stay pi-distributed (chi-square against the erf cell masses), with
  the uniform mu and with a mismatched Gaussian-mixture mu, where the
  independence ratio u(x) / u(y) matters;
* a large step whose proposal density equals the target inside the box has
  acceptance ratio exactly 1;
* the large-step share is l (binomial);
* the ergodic average after a burn-in matches the erf closed form;
* Theorem B of the supplement: with c_tilde >= l / 2 the restore process
  has a time-average variance constant no larger than that of M^l.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import truth
from tests import helpers as H
from workloads import gmm_iso_2d

P_MIN = 1e-4
ELL = 0.3   # the large-step probability of the paper's MH baselines (Sec. 8)


def _run_transitions(prob, x, n_steps, step0=1):
    n = x.shape[0]
    st = O.States(x.copy(), np.zeros(n), np.zeros(n), np.zeros_like(x))
    chains = np.arange(n)
    flags_all = []
    for s in range(n_steps):
        st, dt, flags, _ = O.transitions(prob, st, step0 + s, chains, recompute=(s == 0))
        flags_all.append(flags)
    return st, np.stack(flags_all)


def _mismatched_mu():
    """A two-component diagonal mixture unrelated to the target's modes,
    with a defensive uniform share: u varies strongly over the box."""
    return {"logits": np.log([0.7, 0.3]),
            "means": np.array([[0.3, 0.7], [0.8, 0.2]]),
            "log_std": np.log(np.array([[0.15, 0.2], [0.05, 0.08]])),
            "beta": 0.2}


def _target_as_mu(wl):
    """mu with the target's own mixture (untruncated, no defensive share):
    u = p everywhere inside the box."""
    p = wl.params
    sig = np.asarray(p["sigmas"], dtype=np.float64)
    return {"logits": np.log(p["weights"]), "means": np.asarray(p["means"]).reshape(wl.K, wl.d),
            "log_std": np.log(np.repeat(sig[:, None], wl.d, axis=1)), "beta": 0.0}


@pytest.mark.parametrize("local,step,mu", [("rwmh", 0.05, None), ("mala", 0.03, None),
                                           ("rwmh", 0.05, "mismatched")])
def test_mixture_kernel_is_pi_invariant(oracle_lib, local, step, mu):
    wl = gmm_iso_2d()
    rng = np.random.default_rng(41)
    n = 60000
    x0 = H.sample_pi_iso(wl, n, rng)
    prob = O.Problem(wl, c_tilde=0.0, step=step, local=local, large_step_prob=ELL,
                     mu=_mismatched_mu() if mu else None)
    st, flags = _run_transitions(prob, x0, 40)
    assert not np.any(flags & O.FLAG_KILL)
    # the large steps did move chains (so the check is not of K_0 alone)
    assert np.count_nonzero(((flags & O.FLAG_LARGE) != 0) & ((flags & O.FLAG_ACCEPT) != 0)) > 0.02 * n
    edges = np.linspace(0, 1, 11)
    obs = H.hist2d(st.x, edges).ravel()
    exp_ = H.iso_cell_masses(wl, edges).ravel()
    exp_ = exp_ / exp_.sum()
    assert H.chi2_pvalue(obs, exp_ * n) > P_MIN


def test_large_step_share_is_l(oracle_lib):
    wl = gmm_iso_2d()
    n, steps = 20000, 10
    x0 = H.sample_pi_iso(wl, n, np.random.default_rng(42))
    prob = O.Problem(wl, c_tilde=0.0, large_step_prob=ELL)
    _, flags = _run_transitions(prob, x0, steps)
    k = np.count_nonzero(flags & O.FLAG_LARGE)
    N = flags.size
    z = (k - N * ELL) / math.sqrt(N * ELL * (1 - ELL))
    assert abs(z) < 4.0
    # l = 0: no large steps, and the same trajectory as the small-step chain
    a, fa = _run_transitions(O.Problem(wl, c_tilde=0.0, large_step_prob=0.0), x0[:2000], steps)
    b, fb = _run_transitions(O.Problem(wl, c_tilde=0.0), x0[:2000], steps)
    assert not np.any(fa & O.FLAG_LARGE)
    assert np.array_equal(fa, fb) and np.array_equal(a.x, b.x)


def test_large_step_with_proposal_equal_to_target_always_accepted(oracle_lib):
    """l = 1 and u = p inside the box: the ratio p(y) u(x) / (p(x) u(y)) is
    1, so every in-box proposal is accepted and every proposal outside the
    box (p = 0 there) is rejected."""
    wl = gmm_iso_2d()
    # one mode moved next to the edge, so that proposals leave the box
    wl.params = dict(wl.params)
    wl.params["means"] = np.array(wl.params["means"], dtype=np.float64)
    wl.params["means"][0] = [0.03, 0.5]
    n = 20000
    x0 = H.sample_pi_iso(wl, n, np.random.default_rng(43))
    prob = O.Problem(wl, c_tilde=0.0, large_step_prob=1.0, mu=_target_as_mu(wl))
    _, flags = _run_transitions(prob, x0, 5)
    assert np.all(flags & O.FLAG_LARGE)
    outside = (flags & O.FLAG_OUTSIDE) != 0
    accepted = (flags & O.FLAG_ACCEPT) != 0
    assert np.any(outside) and np.any(accepted)
    assert np.array_equal(accepted, ~outside)


@pytest.mark.parametrize("rb", [False, True])
def test_mh_ergodic_average_matches_erf_truth(oracle_lib, rb):
    """M^l with a burn-in: the pooled ergodic average of f = p over
    independent chains estimates pi f = int p^2 / int p.  With the
    conditional-mean holding time (rb) every step weighs 1, the discrete-time
    average of the paper's MH baselines."""
    wl = gmm_iso_2d()
    C, burn, n = 512, 2000, 6000
    prob = O.Problem(wl, c_tilde=0.0, large_step_prob=ELL, burn_in=burn, rb_dt=rb)
    r = O.run(prob, 0, C, n_steps=burn + n)
    est = O.estimate(r)
    tr = truth.truths(wl)
    assert est["tours_done"] == 0 and est["tours_censored"] == 0
    assert math.isnan(est["p_lambda"]) and math.isnan(est["lam_pf"])
    assert est["transitions"] == C * n
    assert abs(est["large_steps"] / est["transitions"] - ELL) < 0.01
    if rb:
        assert np.all(r.t_done == n)
    assert abs(est["pi_f"] - tr["pi_f"]) < 3 * est["pi_f_se"]


def _sigma2(r):
    """Variance constant of the time average of f = p and its standard
    error over chains (a ratio of sums, delta method)."""
    A, T = np.asarray(r.a_done), np.asarray(r.t_done)
    R = A.sum() / T.sum()
    e = (A - R * T) ** 2
    s2, se = O._ratio(e, T)
    assert abs(s2 - O.asymptotic_variance(r)) < 1e-9 * s2
    return s2, se


def test_theorem_b_ordering_of_variance_constants(oracle_lib):
    """Theorem B of the supplement: if c_tilde >= l / 2 (p_lambda-scaled
    constant of the killing rate), the restore process built on the small
    step kernel and mu has a time-average variance constant for bounded f
    no larger than that of the MH chain M^l with the same two kernels (as
    a continuous-time process with unit-rate holding times, i.e. generator
    K_l - id).  Checked at c_tilde = l / 2 and at the paper's c_tilde = 1,
    for f = p on the 2-D mixture, with a 3-SE allowance."""
    wl = gmm_iso_2d()
    C = 2048
    mh = O.run(O.Problem(wl, c_tilde=0.0, large_step_prob=ELL, burn_in=2000), 0, C, n_steps=2000 + 8000)
    s_mh, se_mh = _sigma2(mh)
    for ct in (ELL / 2, 1.0):
        rs = O.run(O.Problem(wl, c_tilde=ct), 0, C, n_steps=2000)
        est = O.estimate(rs)
        assert est["tours_censored"] == 0
        s_r, se_r = _sigma2(rs)
        assert s_r < s_mh + 3 * math.hypot(se_r, se_mh), (ct, s_r, s_mh)
    # at c_tilde = 1 the restore constant is well below (not just within noise)
    assert s_r < 0.6 * s_mh
