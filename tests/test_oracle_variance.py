"""Pins of the oracle's time-average variance constant -- no GPU.

`oracle.asymptotic_variance` estimates sigma^2 with
Var(int_0^t f ds / t) ~ sigma^2 / t, the quantity Theorem B of the
supplement orders (Dirichlet forms order the variance constants of time
averages).  Two facts that do not come from the estimator's own formula
pin it:

* Zero local step (sigma = 0): a tour stays at its start x ~ mu for
  tau ~ Exp(k(x)), k = c~ u / p (Sec. 6.2, eq. (killing-rate-simplified)),
  so the regenerative constant E[(A - pi f tau)^2] / E[tau] has the closed
  form 2 int (f - pi f)^2 p^2 / u dlambda / (c~ p_lambda) (E[tau^2 | x] =
  2 / k^2, E[tau] = p_lambda / c~; u = 1 on the box).  The integral is
  taken by 400^2 Gauss-Legendre on the box and checked at two c~ whose mean
  lifetimes p_lambda / c~ differ sixteenfold, so a wrong time scale (tours
  in place of time, say) cannot pass both.
* The MH chain M^l (Sec. 5, eq. (mixture-proposal-kernel)): over
  independent replicates of a whole run, the spread of the pooled time
  average pi f is what the variance constant predicts,
  Var(pi f estimate) = sigma^2 / sum T; the ratio of the two is checked
  against the chi-square law of a sample variance.
"""
import inspect
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from oracle import truth
from workloads import gmm_iso_2d

ELL = 0.3   # the paper's large-step probability for its MH baselines (Sec. 8)


def _zero_step_sigma2_truth(wl, c_tilde: float) -> float:
    """2 int (p - pi p)^2 p^2 dlambda / (c~ p_lambda) on the unit box (f = p,
    u = 1), with pi p = int p^2 / int p, by 400^2 Gauss-Legendre and the
    scipy mixture density (no oracle code)."""
    g, gw = np.polynomial.legendre.leggauss(400)
    xs, ws = (g + 1) / 2, gw / 2
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], 1)
    w = np.asarray(wl.params["weights"])
    m = np.asarray(wl.params["means"])
    s = np.asarray(wl.params["sigmas"])
    p = sum(w[k] * stats.multivariate_normal(m[k], s[k] ** 2 * np.eye(2)).pdf(pts) for k in range(len(w)))
    p = p.reshape(X.shape)
    wgt = np.outer(ws, ws)
    p_lambda = (p * wgt).sum()
    pi_f = (p * p * wgt).sum() / p_lambda
    return float(2.0 * ((p - pi_f) ** 2 * p * p * wgt).sum() / (c_tilde * p_lambda))


def _group_se(fn, r, groups: int = 32) -> float:
    """Standard error of fn(run) from its spread over disjoint chain groups."""
    n = len(r.n_done)
    vals = []
    for g in range(groups):
        sl = slice(g * n // groups, (g + 1) * n // groups)
        sub = O.RunResult(r.n_done[sl], r.t_done[sl], r.a_done[sl], r.censored[sl], r.t_censored[sl],
                          r.transitions[sl], r.accepts[sl], r.kills[sl], None, r.c_tilde)
        vals.append(fn(sub))
    return float(np.std(vals, ddof=1) / math.sqrt(groups))


def check_zero_step_closed_form(av) -> None:
    wl = gmm_iso_2d()
    for c in (0.25, 4.0):
        prob = O.Problem(wl, c_tilde=c, step=0.0)
        r = O.run(prob, 0, 8192, n_steps=800, drain_cap=20000)
        assert r.censored.sum() == 0
        got = av(r)
        want = _zero_step_sigma2_truth(wl, c)
        se = _group_se(av, r)
        assert abs(got - want) < 4 * se, (c, got, want, se)
        # the allowance is a few percent of the value, far below the factor
        # p_lambda / c~ (4 or 1/4) of a wrong time scale
        assert se < 0.05 * want, (c, se, want)


def check_mh_replicate_spread(av) -> None:
    wl = gmm_iso_2d()
    reps, C, burn, n = 48, 256, 1000, 4000
    pif, s2, tot = [], [], []
    for i in range(reps):
        prob = O.Problem(wl, c_tilde=0.0, large_step_prob=ELL, burn_in=burn, rb_dt=True, seed=7100 + 13 * i)
        r = O.run(prob, 0, C, n_steps=burn + n)
        pif.append(r.a_done.sum() / r.t_done.sum())
        s2.append(av(r))
        tot.append(r.t_done.sum())
    pif, s2, tot = np.asarray(pif), np.asarray(s2), np.asarray(tot)
    assert np.all(tot == C * n)                       # unit holding times
    predicted_var = s2.mean() / tot[0]
    q = (reps - 1) * pif.var(ddof=1) / predicted_var  # ~ chi^2_{reps-1}
    lo, hi = stats.chi2.ppf(5e-4, reps - 1), stats.chi2.ppf(1 - 5e-4, reps - 1)
    assert lo < q < hi, (q, lo, hi)


def test_variance_constant_zero_step_closed_form(oracle_lib):
    check_zero_step_closed_form(O.asymptotic_variance)


def test_variance_constant_predicts_replicate_spread_of_mh(oracle_lib):
    check_mh_replicate_spread(O.asymptotic_variance)


def test_zero_step_truth_against_direct_sampling():
    """The closed form itself, against plain Monte Carlo of its definition:
    x ~ U(box), tau ~ Exp(c~ / p(x)), sigma^2 = E[tau^2 (p - pi p)^2] / E[tau]."""
    wl = gmm_iso_2d()
    rng = np.random.default_rng(11)
    n, c = 4_000_000, 4.0
    x = rng.random((n, 2))
    w = np.asarray(wl.params["weights"])
    m = np.asarray(wl.params["means"])
    s = np.asarray(wl.params["sigmas"])
    p = sum(w[k] * stats.multivariate_normal(m[k], s[k] ** 2 * np.eye(2)).pdf(x) for k in range(len(w)))
    tau = rng.exponential(p / c)
    pi_f = truth.truths(wl)["pi_f"]
    y = tau * tau * (p - pi_f) ** 2
    want = _zero_step_sigma2_truth(wl, c)
    got = y.mean() / tau.mean()
    se = y.std() / math.sqrt(n) / tau.mean()
    assert abs(got - want) < 4 * se + 1e-3 * want, (got, want, se)


# plausible mistakes in the estimator, planted in a copy of its source
VARIANCE_MUTATIONS = {
    # normalised per tour instead of per unit of process time
    "per_tour_not_per_time": ("return float((res * res).sum() / T.sum())",
                              "return float((res * res).sum() / np.asarray(r.n_done, dtype=np.float64).sum())"),
    # residuals not centred on the pooled ratio
    "uncentred_residuals": ("res = A - R * T", "res = A"),
    # mean over chains in place of the per-time normalisation
    "mean_over_chains": ("return float((res * res).sum() / T.sum())", "return float((res * res).mean())"),
    # the constant off by a factor of two
    "twice_the_constant": ("return float((res * res).sum() / T.sum())",
                           "return float(2.0 * (res * res).sum() / T.sum())"),
}


@pytest.mark.parametrize("name", sorted(VARIANCE_MUTATIONS))
def test_planted_variance_mistake_is_caught(name, oracle_lib):
    old, new = VARIANCE_MUTATIONS[name]
    src = inspect.getsource(O.asymptotic_variance)
    assert src.count(old) == 1, name
    ns = dict(vars(O))
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    mutant = ns["asymptotic_variance"]
    caught = 0
    for check in (check_zero_step_closed_form, check_mh_replicate_spread):
        try:
            with np.errstate(all="ignore"):
                check(mutant)
        except AssertionError:
            caught += 1
    assert caught > 0, f"no pin caught the planted mistake {name}"
