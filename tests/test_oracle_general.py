"""Pins of the oracle's restore process with local dynamics that are not
pi-invariant -- no GPU.

The local process is the unadjusted random-walk jump process: at rate 1 it
jumps x -> x + sigma z, z ~ N(0, I), with no acceptance test.  Its adjoint
generator applied to p is L* p = Q^T p - p with
(Q^T p)(x) = int_box p(y) N(x; y, sigma^2 I) dy, and the killing rate of
Sec. 6.2, eq. (killing-rate), for a state-independent mu of density u is
k = (c_tilde u + L* p) / p (non-negative only for c_tilde >= sup (p - Q^T p)/u).

Pinned against facts the oracle does not compute itself: Q^T p against
tensor Gauss-Legendre quadrature of its defining integral (densities from
scipy), its total mass against the erf box mass, its small-jump limit
against the closed-form Laplacian of the mixture, the kill law at fixed
states against the quadrature rate, and whole runs against the erf truths
(a wrong rate breaks pi-invariance and biases them).
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as O
from oracle import truth
from tests.test_oracle_pins import P_MIN, _scipy_log_mixture
from workloads import gmm_iso_2d, gmm_iso_2d_unadjusted


def _gl_nodes(lo, hi, panels, order=8):
    """Composite Gauss-Legendre nodes and weights on [lo, hi]."""
    t, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(lo, hi, panels + 1)
    a, b = edges[:-1, None], edges[1:, None]
    x = (0.5 * (b - a) * t[None, :] + 0.5 * (a + b)).ravel()
    ww = (0.5 * (b - a) * w[None, :]).ravel()
    return x, ww


def _inflow_quadrature(wl, sigma, pts):
    """(Q^T p)(x) = int_[0,1]^2 p(y) N(x; y, sigma^2 I) dy by composite
    Gauss-Legendre (panels of sigma / 4)."""
    g, w = _gl_nodes(0.0, 1.0, int(math.ceil(4 / sigma)))
    Y0, Y1 = np.meshgrid(g, g, indexing="ij")
    W = np.outer(w, w)
    py = np.exp(_scipy_log_mixture(wl, np.stack([Y0.ravel(), Y1.ravel()], axis=1))).reshape(Y0.shape)
    out = []
    for x in pts:
        k = np.exp(-((x[0] - Y0) ** 2 + (x[1] - Y1) ** 2) / (2 * sigma * sigma)) / (2 * math.pi * sigma * sigma)
        out.append((W * py * k).sum())
    return np.array(out)


def _probe_points(wl):
    m = wl.params["means"]
    return np.array([m[0], m[1] + 0.03, m[3] - [0.02, 0.05], [0.5, 0.5], [0.0, 0.3], [0.97, 1.0],
                     [0.01, 0.02], [1.0, 1.0], [0.3, 0.999]])


def test_inflow_matches_quadrature(oracle_lib):
    """The erf closed form of Q^T p against quadrature of its definition,
    at the modes, in between, and on the edges and corners of the box
    (where the truncation of p matters)."""
    wl = gmm_iso_2d_unadjusted()
    prob = O.Problem(wl)
    pts = _probe_points(wl)
    for sigma in (0.02, 0.05):
        q = np.exp(O.log_inflow(prob, pts, sigma))
        ref = _inflow_quadrature(wl, sigma, pts)
        np.testing.assert_allclose(q, ref, rtol=1e-9, atol=1e-12)


def test_inflow_conserves_mass(oracle_lib):
    """int Q^T p over the whole plane equals p_lambda (the jump kernel
    moves mass without creating or destroying it, i.e. int L* p = 0, the
    condition of Theorem A of the supplement); the erf box mass is the
    truth.  Q^T p is integrated beyond the box, where jumps land."""
    wl = gmm_iso_2d_unadjusted()
    prob = O.Problem(wl)
    s = wl.step
    g, w = _gl_nodes(-12 * s, 1 + 12 * s, int(math.ceil((1 + 24 * s) / (0.5 * s))), order=6)
    X0, X1 = np.meshgrid(g, g, indexing="ij")
    q = np.exp(O.log_inflow(prob, np.stack([X0.ravel(), X1.ravel()], axis=1))).reshape(X0.shape)
    total = (np.outer(w, w) * q).sum()
    assert abs(total / truth.truths(wl)["p_lambda"] - 1) < 1e-8


def test_small_jumps_give_half_the_laplacian(oracle_lib):
    """Far from the edges, Q^T p - p = (sigma^2 / 2) Laplacian(p) + O(sigma^4)
    (heat kernel).  The Laplacian of the isotropic mixture in closed form:
    sum_k w_k N_k(x) (|x - m_k|^2 / s_k^4 - d / s_k^2)."""
    wl = gmm_iso_2d_unadjusted()
    prob = O.Problem(wl)
    m, w, sg = wl.params["means"], wl.params["weights"], wl.params["sigmas"]
    rng = np.random.default_rng(31)
    x = np.clip(m[rng.integers(0, 4, 12)] + 0.04 * rng.standard_normal((12, 2)), 0.3, 0.7)
    lap = np.zeros(len(x))
    for k in range(4):
        r2 = ((x - m[k]) ** 2).sum(axis=1)
        nk = np.exp(-r2 / (2 * sg[k] ** 2)) / (2 * math.pi * sg[k] ** 2)
        lap += w[k] * nk * (r2 / sg[k] ** 4 - 2 / sg[k] ** 2)
    p = np.exp(_scipy_log_mixture(wl, x))
    sigma = 2e-3
    q = np.exp(O.log_inflow(prob, x, sigma))
    got = (q - p) / (0.5 * sigma * sigma)
    scale = np.abs(lap).max()
    np.testing.assert_allclose(got, lap, rtol=0, atol=5e-3 * scale)
    # the cached density: u_eff = u + (Q^T p - p) / c_tilde
    prob_s = O.Problem(wl, step=sigma)
    ue = np.exp(O.log_u_eff(prob_s, x))
    np.testing.assert_allclose(ue, 1.0 + (q - p) / wl.c_tilde, rtol=1e-12)


@pytest.mark.parametrize("where", ["mode", "shoulder", "tail"])
def test_kill_law_uses_the_general_rate(oracle_lib, where):
    """At a fixed x: P(kill) = k / (1 + k) and dt ~ Exp(1 + k) with
    k = (c_tilde + Q^T p - p) / p from quadrature; the local jump is always
    taken (ACCEPT whenever not killed) and lands at x + sigma z."""
    wl = gmm_iso_2d_unadjusted()
    m = wl.params["means"]
    x = {"mode": m[0], "shoulder": m[0] + 0.06, "tail": m[0] + [0.1, 0.0]}[where]
    p = math.exp(_scipy_log_mixture(wl, x[None])[0])
    q = _inflow_quadrature(wl, wl.step, x[None])[0]
    k = (wl.c_tilde + q - p) / p
    prob = O.Problem(wl)
    n = 60000
    st = O.States(np.tile(x, (n, 1)), np.zeros(n), np.zeros(n), np.zeros((n, 2)))
    new, dt, flags, _ = O.transitions(prob, st, np.arange(n), np.full(n, 9))
    kill = (flags & O.FLAG_KILL) != 0
    pk = k / (1 + k)
    assert abs(kill.mean() - pk) < 4 * math.sqrt(pk * (1 - pk) / n)
    assert stats.kstest(dt * (1 + k), "expon").pvalue > P_MIN
    moved = ~kill
    assert np.all((flags[moved] & O.FLAG_ACCEPT) != 0) and not np.any(flags[kill] & O.FLAG_ACCEPT)
    z = (new.x[moved] - x) / wl.step
    assert stats.kstest(z.ravel(), "norm").pvalue > P_MIN
    assert not np.any(flags & O.FLAG_NEGATIVE_RATE)


def test_jump_off_the_box_is_killed_at_once(oracle_lib):
    """A jump that leaves the box lands where p = 0: the next step kills
    with dt = 0, and the chain regenerates inside.  (A mode moved next to
    the edge, so that jumps from it leave the box often.)"""
    wl = gmm_iso_2d_unadjusted()
    params = dict(wl.params)
    params["means"] = wl.params["means"].copy()
    params["means"][0] = [0.03, 0.5]
    prob = O.Problem(wl.with_(params=params), c_tilde=50.0)
    n = 20000
    x = np.tile([0.01, 0.5], (n, 1))
    st = O.States(x, np.zeros(n), np.zeros(n), np.zeros((n, 2)))
    new, _, flags, _ = O.transitions(prob, st, np.arange(n), np.full(n, 3))
    out = (flags & O.FLAG_OUTSIDE) != 0
    assert out.sum() > 1000 and np.all(new.lp[out] == -np.inf)
    sub = O.States(new.x[out], new.lp[out], new.lu[out], new.g[out])
    nxt, dt, fl2, _ = O.transitions(prob, sub, 7, np.arange(out.sum()), recompute=False)
    assert np.all(fl2 & O.FLAG_KILL) and np.all(dt == 0.0) and np.all(np.isfinite(nxt.lp))


def test_whole_run_matches_erf_truth(oracle_lib):
    """The general restore process is pi-invariant, so its tour-ratio
    estimates are consistent: p_lambda, lambda(p f) and pi f within 4 SE of
    the erf closed forms, no censored tour, no negative rate."""
    wl = gmm_iso_2d_unadjusted()
    r = O.run(O.Problem(wl), 0, wl.n_chains)
    est = O.estimate(r)
    tr = truth.truths(wl)
    assert est["nonfinite"] == 0 and est["tours_censored"] == 0
    for key in ("p_lambda", "lam_pf", "pi_f"):
        assert abs(est[key] - tr[key]) < 4 * est[key + "_se"], (key, est[key], tr[key], est[key + "_se"])
    # every non-kill step is a taken jump
    assert abs(est["accept_rate"] + est["kill_rate"] - 1) < 1e-12


def test_negative_rate_marks_the_chain(oracle_lib):
    """With c_tilde below sup (p - Q^T p) the rate is negative at the
    modes: u_eff is NaN there, a step from such a state is flagged, its dt
    is NaN, and whole runs report the affected chains as non-finite."""
    wl = gmm_iso_2d_unadjusted().with_(c_tilde=1.0)
    prob = O.Problem(wl)
    m = wl.params["means"][0][None]
    assert np.isnan(O.log_u_eff(prob, m)[0])
    st = O.States(np.tile(m, (8, 1)), np.zeros(8), np.zeros(8), np.zeros((8, 2)))
    _, dt, flags, _ = O.transitions(prob, st, np.arange(8), np.zeros(8))
    assert np.all(flags & O.FLAG_NEGATIVE_RATE) and np.all(np.isnan(dt))
    est = O.estimate(O.run(prob, 0, 512, n_steps=200, drain_cap=800))
    assert est["nonfinite"] > 0
    # with the rule's c_tilde the same state is fine
    assert np.isfinite(O.log_u_eff(O.Problem(gmm_iso_2d_unadjusted()), m)[0])


def test_unadjusted_needs_the_isotropic_mixture_and_killing(oracle_lib):
    wl = gmm_iso_2d_unadjusted()
    with pytest.raises(ValueError):
        O.Problem(wl, c_tilde=0.0)
    with pytest.raises(ValueError):
        O.Problem(wl, large_step_prob=0.3)
    # the invariant kernel on the same target is unaffected
    assert O.Problem(gmm_iso_2d()).local.kind == O.LOCAL_RWMH
