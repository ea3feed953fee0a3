"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics -- no GPU.

Each statistical test uses fixed seeds (so it is deterministic) and a
threshold of p > 1e-4 (z < 4) per check; across the ~30 checks of this file
that is a family-wise false-alarm rate below 1e-2 for a fresh seed choice.
"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from oracle import truth
from tests import helpers as H
from workloads import gmm_full, gmm_iso_2d, one_d_three_mode

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
P_MIN = 1e-4


# ---------------------------------------------------------------------------
# random numbers
# ---------------------------------------------------------------------------

def _kat_rows():
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v, 16) for v in line.split()])
    return rows


def test_philox_known_answers(oracle_lib):
    for row in _kat_rows():
        assert list(O.philox(row[0:4], row[4:6])) == row[6:10]


def test_philox_matches_rocrand(oracle_lib, tmp_path):
    """rocRAND's open-source Philox4x32-10 (ROCm headers), compiled for the
    host, must agree bit for bit on random counters and keys."""
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "probe"
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-I/opt/rocm/include",
                    os.path.join(ROOT, "tests", "pins", "rocrand_philox_probe.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    rng = np.random.default_rng(7)
    vals = rng.integers(0, 2 ** 32, size=(200, 6), dtype=np.uint64)
    inp = "\n".join(" ".join(f"{int(v):x}" for v in row) for row in vals) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for row, line in zip(vals, out):
        ref = [int(v, 16) for v in line.split()]
        assert list(O.philox(row[:4], row[4:6])) == ref


def test_uniform_mapping_exact_in_fp32(oracle_lib):
    rs = [0, 1, 511, 512, 2 ** 31, 2 ** 32 - 1, 123456789]
    for r in rs:
        u = O.u01(r)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
        assert u == (2 * (r >> 9) + 1) / 2 ** 24
    assert O.u01(0) == 2.0 ** -24
    assert O.u01(2 ** 32 - 1) == 1 - 2.0 ** -24


def test_normals_and_exponentials_from_steps(oracle_lib):
    """The step's Box-Muller normals (seen through sigma-scaled random-walk
    proposals from a fixed x with every move accepted, c_tilde = 0) are
    standard normal; -ln u of the holding clock is Exp(1)."""
    wl = gmm_iso_2d()
    # a nearly flat target so every proposal inside the box is accepted
    flat = wl.with_(params={"weights": np.array([1.0]), "means": np.array([[0.5, 0.5]]),
                            "sigmas": np.array([1e3])}, K=1)
    prob = O.Problem(flat, c_tilde=0.0, step=1e-3)
    n = 40000
    st = O.States(np.full((n, 2), 0.5), np.zeros(n), np.zeros(n), np.zeros((n, 2)))
    new, dt, flags, _ = O.transitions(prob, st, np.arange(n), np.full(n, 3))
    assert np.all(flags & O.FLAG_ACCEPT)
    z = (new.x - 0.5) / 1e-3
    for i in range(2):
        assert stats.kstest(z[:, i], "norm").pvalue > P_MIN
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 4 / math.sqrt(n)
    assert stats.kstest(dt, "expon").pvalue > P_MIN


# ---------------------------------------------------------------------------
# densities
# ---------------------------------------------------------------------------

def _scipy_log_mixture(wl, x):
    w = wl.params["weights"]
    m = wl.params["means"]
    if wl.target == "gmm_iso":
        covs = [np.eye(wl.d) * s * s for s in wl.params["sigmas"]]
    else:
        covs = wl.params["covs"]
    comps = np.stack([np.log(w[k]) + np.atleast_1d(stats.multivariate_normal(m[k], covs[k]).logpdf(x))
                      for k in range(wl.K)], axis=-1)
    from scipy.special import logsumexp
    return logsumexp(comps, axis=-1)


@pytest.mark.parametrize("make", [gmm_iso_2d, gmm_full])
def test_log_target_matches_scipy(oracle_lib, make):
    wl = make()
    prob = O.Problem(wl)
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.uniform(0, 1, (200, wl.d)), wl.params["means"]])
    lp = O.log_target(prob, x)
    ref = _scipy_log_mixture(wl, x)
    np.testing.assert_allclose(lp, ref, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("make", [gmm_iso_2d, gmm_full])
def test_grad_log_target_central_differences(oracle_lib, make):
    wl = make()
    prob = O.Problem(wl)
    rng = np.random.default_rng(12)
    m = wl.params["means"]
    x = np.clip(m[rng.integers(0, wl.K, 20)] + 0.01 * rng.standard_normal((20, wl.d)), 0.01, 0.99)
    _, g = O.log_target(prob, x, grad=True)
    h = 1e-6
    for i in range(wl.d):
        e = np.zeros(wl.d)
        e[i] = h
        fd = (O.log_target(prob, x + e) - O.log_target(prob, x - e)) / (2 * h)
        np.testing.assert_allclose(g[:, i], fd, rtol=1e-5, atol=1e-4 * np.abs(fd).max())


def test_log_target_zero_outside_box(oracle_lib):
    prob = O.Problem(gmm_iso_2d())
    lp = O.log_target(prob, np.array([[-1e-9, 0.5], [0.5, 1 + 1e-9], [0.0, 1.0]]))
    assert lp[0] == -np.inf and lp[1] == -np.inf and np.isfinite(lp[2])


# ---------------------------------------------------------------------------
# truths
# ---------------------------------------------------------------------------

def test_iso_truth_matches_quadrature():
    wl = gmm_iso_2d()
    tr = truth.truths(wl)
    g, gw = np.polynomial.legendre.leggauss(400)
    pts, w = (g + 1) / 2, gw / 2
    X, Y = np.meshgrid(pts, pts, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel()], 1)
    p = np.exp(_scipy_log_mixture(wl, x)).reshape(X.shape)
    W2 = np.outer(w, w)
    assert abs((p * W2).sum() - tr["p_lambda"]) < 1e-10
    assert abs((p * p * W2).sum() / tr["lam_pf"] - 1) < 1e-10


def test_full_truth_matches_iid_sampling():
    """Box probabilities from the Genz routine against plain Monte Carlo
    (component draws counted inside the box)."""
    wl = gmm_full()
    tr = truth.truths(wl)
    rng = np.random.default_rng(13)
    n = 400000
    w, m, c = wl.params["weights"], wl.params["means"], wl.params["covs"]
    inside = 0.0
    for k in range(wl.K):
        x = rng.multivariate_normal(m[k], c[k], size=n)
        inside += w[k] * np.all((x >= 0) & (x <= 1), axis=1).mean()
    se = math.sqrt(0.25 / n)
    assert abs(inside - tr["p_lambda"]) < 4 * se
    # int p^2 = E_pi[p] p_lambda: estimate from exact draws of pi
    k = rng.choice(wl.K, size=n, p=w)
    x = np.array([rng.multivariate_normal(m[j], c[j]) for j in k[:60000]])
    x = x[np.all((x >= 0) & (x <= 1), axis=1)]
    px = np.exp(_scipy_log_mixture(wl, x))
    est = px.mean() * tr["p_lambda"]
    assert abs(est - tr["lam_pf"]) < 4 * px.std() / math.sqrt(len(px)) * tr["p_lambda"]


# ---------------------------------------------------------------------------
# the step: invariance of nu = p + c_tilde u (pure-jump transition rule)
# ---------------------------------------------------------------------------

def _sample_nu(wl, c_tilde, n, rng):
    """nu ~ (p + c_tilde u) / (p_lambda + c_tilde) with u uniform on the box."""
    pl = truth.truths(wl)["p_lambda"]
    from_pi = rng.uniform(size=n) < pl / (pl + c_tilde)
    x = rng.uniform(size=(n, wl.d))
    x[from_pi] = H.sample_pi_iso(wl, int(from_pi.sum()), rng)
    return x, pl


def _run_transitions(prob, x, n_steps, step0=1):
    n = x.shape[0]
    st = O.States(x.copy(), np.zeros(n), np.zeros(n), np.zeros_like(x))
    chains = np.arange(n)
    first = None
    for s in range(n_steps):
        st, dt, flags, _ = O.transitions(prob, st, step0 + s, chains, recompute=(s == 0))
        if first is None:
            first = (dt, flags)
    return st, first


@pytest.mark.parametrize("local,step,c_tilde", [("rwmh", 0.05, 1.0), ("mala", 0.03, 1.0),
                                                ("rwmh", 0.05, 4.0)])
def test_jump_chain_leaves_nu_invariant(oracle_lib, local, step, c_tilde):
    """The embedded jump chain of the restore process has transition
    (1/(1+k)) zeta + (k/(1+k)) mu; with k = c_tilde u / p it leaves
    nu = p + c_tilde u invariant.  Start from exact nu draws, take 30
    transitions, compare a 10x10 histogram with nu's cell masses; also the
    first step's kill probability c_tilde / (p_lambda + c_tilde), mean
    holding time p_lambda / (p_lambda + c_tilde) and mean dt p(x_{i-1}) =
    lambda(p^2) / (p_lambda + c_tilde)."""
    wl = gmm_iso_2d()
    rng = np.random.default_rng(21)
    n = 60000
    x0, pl = _sample_nu(wl, c_tilde, n, rng)
    prob = O.Problem(wl, c_tilde=c_tilde, step=step, local=local)
    st, (dt, flags) = _run_transitions(prob, x0, 30)
    edges = np.linspace(0, 1, 11)
    obs = H.hist2d(st.x, edges).ravel()
    exp_ = (H.iso_cell_masses(wl, edges) + c_tilde * 0.01).ravel() / (pl + c_tilde)
    assert H.chi2_pvalue(obs, exp_ * n) > P_MIN
    Z = pl + c_tilde
    kill = (flags & O.FLAG_KILL) != 0
    pk = c_tilde / Z
    assert abs(kill.mean() - pk) < 4 * math.sqrt(pk * (1 - pk) / n)
    assert abs(dt.mean() - pl / Z) < 4 * dt.std() / math.sqrt(n)
    px = np.exp(_scipy_log_mixture(wl, x0))
    lpf = truth.truths(wl)["lam_pf"]
    v = dt * px
    assert abs(v.mean() - lpf / Z) < 4 * v.std() / math.sqrt(n)


@pytest.mark.parametrize("xpt", [(0.5, 0.5), "mode", (0.05, 0.95)])
def test_kill_and_clock_law_at_fixed_state(oracle_lib, xpt):
    """At a fixed x: P(kill) = k/(1+k), dt ~ Exp(1+k), and dt is independent
    of which clock fired (competing exponentials)."""
    wl = gmm_iso_2d()
    if xpt == "mode":
        xpt = tuple(wl.params["means"][0] + 0.03)
    x = np.array(xpt, dtype=np.float64)
    p = math.exp(_scipy_log_mixture(wl, x[None])[0])
    c_tilde = 2.0
    k = c_tilde * 1.0 / p
    prob = O.Problem(wl, c_tilde=c_tilde)
    n = 60000
    st = O.States(np.tile(x, (n, 1)), np.zeros(n), np.zeros(n), np.zeros((n, 2)))
    _, dt, flags, _ = O.transitions(prob, st, np.arange(n), np.full(n, 5))
    kill = (flags & O.FLAG_KILL) != 0
    pk = k / (1 + k)
    assert abs(kill.mean() - pk) < 4 * math.sqrt(pk * (1 - pk) / n) + 1e-12
    assert stats.kstest(dt * (1 + k), "expon").pvalue > P_MIN
    if 200 < kill.sum() < n - 200:
        assert stats.ks_2samp(dt[kill], dt[~kill]).pvalue > P_MIN


# ---------------------------------------------------------------------------
# lifetimes and special cases
# ---------------------------------------------------------------------------

def _first_tours(prob, n, max_steps=20000):
    """Simulate the first tour of chains 0..n-1: x_0 ~ mu, step until the
    first kill.  Returns (lifetime, number of steps)."""
    st = O.init_states(prob, np.arange(n))
    tau = np.zeros(n)
    steps = np.zeros(n, dtype=np.int64)
    alive = np.ones(n, dtype=bool)
    s = 0
    while alive.any() and s < max_steps:
        idx = np.nonzero(alive)[0]
        sub = O.States(st.x[idx], st.lp[idx], st.lu[idx], st.g[idx])
        sub2, dt, flags, _ = O.transitions(prob, sub, s, idx, recompute=False)
        tau[idx] += dt
        steps[idx] += 1
        st.x[idx], st.lp[idx], st.lu[idx], st.g[idx] = sub2.x, sub2.lp, sub2.lu, sub2.g
        alive[idx[(flags & O.FLAG_KILL) != 0]] = False
        s += 1
    assert not alive.any()
    return tau, steps


def test_expected_lifetime_one_d_example(oracle_lib):
    """E_mu[tau] = 1/c with c_tilde = c p_lambda; the paper's 1-D example
    uses c = 1/4, i.e. an expected tour length of 4
    (tests/golden/worked_example_lifetime.txt)."""
    with open(os.path.join(ROOT, "tests", "golden", "worked_example_lifetime.txt")) as f:
        c, expected = [float(v) for v in next(l for l in f if l.strip() and not l.startswith("#")).split()]
    wl = one_d_three_mode()
    pl = truth.gmm_iso_power_integral(wl, 1)
    prob = O.Problem(wl, c_tilde=c * pl)
    tau, _ = _first_tours(prob, 40000)
    assert abs(tau.mean() - expected) < 4 * tau.std() / math.sqrt(len(tau))


def test_zero_step_reduces_to_randomised_importance_sampling(oracle_lib):
    """With a zero local step the chain never moves within a tour, so the
    lifetime is Exp(k(x)) at x ~ mu: E[c tau] = p_lambda and E[(c tau)^2] =
    2 int p^2 / u (u = 1 on the box)."""
    wl = gmm_iso_2d()
    prob = O.Problem(wl, c_tilde=1.0, step=0.0)
    tau, _ = _first_tours(prob, 60000)
    tr = truth.truths(wl)
    n = len(tau)
    assert abs(tau.mean() - tr["p_lambda"]) < 4 * tau.std() / math.sqrt(n)
    t2 = tau * tau
    assert abs(t2.mean() - 2 * tr["lam_pf"]) < 4 * t2.std() / math.sqrt(n)


def test_zero_step_rao_blackwellised_moments(oracle_lib):
    """With a zero step and the conditional-mean holding time 1/(1+k) in
    place of the sampled one, a tour at x ~ mu lasts Geometric(k/(1+k))
    steps of 1/(1+k) each (k = c/p, u = 1 on the box), so E[c tau] =
    p_lambda is unchanged while E[(c tau)^2] = int p^2 (2p + c)/(p + c):
    between int p^2 (c -> inf) and the sampled 2 int p^2 (c -> 0).  The
    integral by 400^2 Gauss-Legendre on the box."""
    wl = gmm_iso_2d()
    c = 20.0
    prob = O.Problem(wl, c_tilde=c, step=0.0, rb_dt=True)
    tau, _ = _first_tours(prob, 60000)
    tau = c * tau
    g, gw = np.polynomial.legendre.leggauss(400)
    xs, ws = (g + 1) / 2, gw / 2
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    p = np.exp(O.log_target(prob, np.stack([X.ravel(), Y.ravel()], 1))).reshape(X.shape)
    wgt = np.outer(ws, ws)
    m1 = (p * wgt).sum()
    m2 = (p * p * (2 * p + c) / (p + c) * wgt).sum()
    n = len(tau)
    assert abs(tau.mean() - m1) < 4 * tau.std() / math.sqrt(n)
    t2 = tau * tau
    assert abs(t2.mean() - m2) < 4 * t2.std() / math.sqrt(n)
    # the sampled holding time has the larger second moment 2 int p^2
    assert m2 < 2 * (p * p * wgt).sum() - 8 * t2.std() / math.sqrt(n)


def test_constant_rate_when_target_equals_mu(oracle_lib):
    """p proportional to u: k = c is constant, so tour lifetimes are Exp(c)
    and steps per tour are Geometric(c / (1 + c))."""
    wl = gmm_iso_2d().with_(params={"weights": np.array([1.0]), "means": np.array([[0.5, 0.5]]),
                                    "sigmas": np.array([1e3])}, K=1)
    p0 = 1.0 / (2 * math.pi * 1e6)
    c = 0.5
    prob = O.Problem(wl, c_tilde=c * p0)
    tau, steps = _first_tours(prob, 40000)
    assert stats.kstest(tau * c, "expon").pvalue > P_MIN
    q = c / (1 + c)
    kmax = 12
    obs = np.array([(steps == j).sum() for j in range(1, kmax)] + [(steps >= kmax).sum()])
    pr = np.array([q * (1 - q) ** (j - 1) for j in range(1, kmax)] + [(1 - q) ** (kmax - 1)])
    assert H.chi2_pvalue(obs, pr * len(steps)) > P_MIN


@pytest.mark.parametrize("local,step", [("rwmh", 0.05), ("mala", 0.03)])
def test_local_kernel_alone_is_pi_invariant(oracle_lib, local, step):
    """c_tilde = 0 turns off killing: a plain MH chain (Alg. 1), which keeps
    exact pi draws distributed as pi."""
    wl = gmm_iso_2d()
    rng = np.random.default_rng(31)
    n = 60000
    x0 = H.sample_pi_iso(wl, n, rng)
    prob = O.Problem(wl, c_tilde=0.0, step=step, local=local)
    st, (dt, flags) = _run_transitions(prob, x0, 40)
    assert not np.any(flags & O.FLAG_KILL)
    edges = np.linspace(0, 1, 11)
    obs = H.hist2d(st.x, edges).ravel()
    exp_ = H.iso_cell_masses(wl, edges).ravel()
    exp_ = exp_ / exp_.sum()
    assert H.chi2_pvalue(obs, exp_ * n) > P_MIN


# ---------------------------------------------------------------------------
# whole runs against closed forms
# ---------------------------------------------------------------------------

def test_whole_run_2d_matches_erf_closed_form(oracle_lib):
    wl = gmm_iso_2d()
    est = O.estimate(O.run(O.Problem(wl), 0, wl.n_chains))
    tr = truth.truths(wl)
    assert est["tours_censored"] == 0
    for key in ("p_lambda", "lam_pf", "pi_f"):
        assert abs(est[key] - tr[key]) < 3 * est[key + "_se"], key


def test_whole_run_2d_rao_blackwellised_matches_erf_closed_form(oracle_lib):
    """The conditional-mean holding time keeps the whole-run estimates
    unbiased (within 3 SE of the erf truth) and its SE is not larger than
    with the sampled holding time, on the same chains and clocks."""
    wl = gmm_iso_2d()
    est = O.estimate(O.run(O.Problem(wl, rb_dt=True), 0, wl.n_chains))
    ref = O.estimate(O.run(O.Problem(wl), 0, wl.n_chains))
    tr = truth.truths(wl)
    assert est["tours_censored"] == 0 and est["tours_done"] == ref["tours_done"]
    for key in ("p_lambda", "lam_pf", "pi_f"):
        assert abs(est[key] - tr[key]) < 3 * est[key + "_se"], key
        assert est[key + "_se"] <= 1.02 * ref[key + "_se"], key


def test_whole_run_full_cov_mala_2d_matches_genz_truth(oracle_lib):
    """Full-covariance mixture with MALA local moves and uniform mu."""
    from oracle.choose_c_tilde import c_tilde_rule
    wl = gmm_full(d=2, K=4, n_chains=4096, n_steps=1000, problem_seed=77)
    wl = wl.with_(c_tilde=c_tilde_rule(wl))
    est = O.estimate(O.run(O.Problem(wl), 0, wl.n_chains))
    tr = truth.truths(wl)
    assert est["tours_censored"] == 0
    for key in ("p_lambda", "lam_pf", "pi_f"):
        assert abs(est[key] - tr[key]) < 3 * est[key + "_se"], key


mixture_mu_from_target = H.mixture_mu_from_target


def test_whole_run_8d_mixture_mu_matches_genz_truth(oracle_lib):
    """The 8-D, 16-component workload with MALA and a mixture mu (the shape
    of the learned regeneration distribution): estimates within 3 SE of the
    Genz-routine truths."""
    wl = gmm_full(n_chains=4096)
    prob = O.Problem(wl, mu=mixture_mu_from_target(wl), c_tilde=1.0)
    est = O.estimate(O.run(prob, 0, wl.n_chains))
    tr = truth.truths(wl)
    assert est["tours_censored"] == 0
    for key in ("p_lambda", "lam_pf", "pi_f"):
        assert abs(est[key] - tr[key]) < 3 * est[key + "_se"], key


def test_mixture_mu_density_integrates_to_one(oracle_lib):
    """u of the defensive mixture integrates to 1 over R^d (2-D quadrature
    over a box that holds all of the Gaussian mass)."""
    wl = gmm_full(d=2, K=4, problem_seed=77)
    prob = O.Problem(wl, mu=mixture_mu_from_target(wl, beta=0.3))
    g, gw = np.polynomial.legendre.leggauss(300)
    lo, hi = -1.0, 2.0
    pts, w = lo + (hi - lo) * (g + 1) / 2, gw * (hi - lo) / 2
    X, Y = np.meshgrid(pts, pts, indexing="ij")
    lu = O.log_mu(prob, np.stack([X.ravel(), Y.ravel()], 1)).reshape(X.shape)
    # the uniform share has a jump at the box edge: integrate it separately
    inside = (X >= 0) & (X <= 1) & (Y >= 0) & (Y <= 1)
    gauss = np.exp(lu) - 0.3 * inside
    assert abs((gauss * np.outer(w, w)).sum() - 0.7) < 1e-6


def test_standard_error_is_calibrated(oracle_lib):
    """Replicates with independent seeds: their spread matches the reported
    delta-method standard error."""
    wl = gmm_iso_2d(n_chains=256, n_steps=300)
    ests = [O.estimate(O.run(O.Problem(wl, seed=900 + r), 0, 256)) for r in range(24)]
    vals = np.array([e["p_lambda"] for e in ests])
    ses = np.array([e["p_lambda_se"] for e in ests])
    ratio = vals.std(ddof=1) / ses.mean()
    assert 0.6 < ratio < 1.5
    tr = truth.truths(wl)
    assert abs(vals.mean() - tr["p_lambda"]) < 4 * vals.std(ddof=1) / math.sqrt(len(vals))


def test_run_is_deterministic_and_thread_invariant(oracle_lib):
    wl = gmm_iso_2d(n_chains=300, n_steps=100)
    prob = O.Problem(wl)
    a = O.run(prob, 0, 300, threads=1)
    b = O.run(prob, 0, 300, threads=5)
    c = O.run(prob, 100, 300, threads=3)
    np.testing.assert_array_equal(a.t_done, b.t_done)
    np.testing.assert_array_equal(a.n_done[100:], c.n_done)
    np.testing.assert_array_equal(a.a_done[100:], c.a_done)


def test_stored_truths_match_the_oracle():
    """tests/golden/truths.json (read by the benchmark to score estimates)
    is what the oracle's truth routines give today, to the accuracy of
    Genz's randomised rule (its state carries over between calls, so the
    last digits depend on what ran before in the process)."""
    import json
    import os
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    import write_truths
    with open(write_truths.PATH) as f:
        stored = json.load(f)
    # the batched targets: the first, the last and the largest, and a seeded sample
    from workloads import batched_uneven
    ts = batched_uneven()
    big = max(range(len(ts)), key=lambda i: ts[i].d * ts[i].K)
    sample = sorted({0, len(ts) - 1, big, *np.random.default_rng(8).choice(len(ts), 5, replace=False).tolist()})
    fresh = write_truths.compute(uneven_targets=sample)
    stored["batched_uneven"]["p_lambda"] = [stored["batched_uneven"]["p_lambda"][i] for i in sample]
    assert stored.keys() == fresh.keys()
    for name in fresh:
        for k, v in fresh[name].items():
            if k == "tiles":
                np.testing.assert_allclose(stored[name][k], v, rtol=1e-12)
            else:
                assert stored[name][k] == pytest.approx(v, rel=1e-5), (name, k)
