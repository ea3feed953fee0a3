"""Pins of the oracle's rendering-shaped integrand (12-D primary sample
space -> 512x512 image) -- no GPU."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import truth
from workloads import pss_render


@pytest.fixture(scope="module")
def wl():
    return pss_render(n_chains=4096, n_steps=200)


def _g(prob, x):
    return np.exp(O.log_target(prob, x))


def test_texture_and_lobes_normalised(oracle_lib, wl):
    """Each texture integrates to 1 (integer frequencies != 0) and each lobe
    h integrates to 1 over the unit square (vMF normalisation times the 4 pi
    area element of z = 1 - 2u, phi = 2 pi v).  Checked through g itself:
    with the other factors held fixed, integrating over one factor's
    coordinates gives the factor's integral."""
    prob = O.Problem(wl)
    rng = np.random.default_rng(4)
    # tB: vary x6..x11 by Monte Carlo with everything else fixed
    base = np.full(12, 0.37)
    n = 400000
    xs = np.tile(base, (n, 1))
    xs[:, 6:] = rng.uniform(size=(n, 6))
    gv = _g(prob, xs)
    g0 = _g(prob, np.tile(base, (1, 1)))[0]
    # g / tB(base) averaged over x6..11 = g(base) / tB(base) * mean(tB) -> ratio of means
    tb_vals = gv / (g0 / _tb(wl, base[6:]))
    assert abs(tb_vals.mean() - 1.0) < 4 * tb_vals.std() / math.sqrt(n)
    # lobe 2 on (x2, x3): Gauss-Legendre on a fine grid, other coordinates fixed
    k = 2000
    gx, gw = np.polynomial.legendre.leggauss(k)
    u = (gx + 1) / 2
    w = gw / 2
    U, V = np.meshgrid(u, u, indexing="ij")
    pts = np.tile(base, (k * k, 1))
    pts[:, 2] = U.ravel()
    pts[:, 3] = V.ravel()
    gv = _g(prob, pts).reshape(k, k)
    integral = (gv * np.outer(w, w)).sum()
    # integral over (x2,x3) of g = tA tB [b + w1 h1 + w2 * 1 + w3 h3]
    tA, tB = _ta(wl, base[:2]), _tb(wl, base[6:])
    wts = wl.params["lobe_weights"]
    h1 = _lobe(wl, 0, base[0], base[1])
    h3 = _lobe(wl, 2, base[4], base[5])
    expect = tA * tB * (wl.params["base"][0] + wts[0] * h1 + wts[1] + wts[2] * h3)
    assert abs(integral / expect - 1) < 1e-4


def _tex(freq, amp, ph, y):
    return 1 + (amp * np.sin(2 * math.pi * (freq @ y) + ph)).sum() / 8


def _ta(wl, y):
    p = wl.params
    return _tex(p["tex_a_freq"], p["tex_a_amp"], p["tex_a_phase"], y)


def _tb(wl, y):
    p = wl.params
    return _tex(p["tex_b_freq"], p["tex_b_amp"], p["tex_b_phase"], y)


def _lobe(wl, l, u, v):
    p = wl.params
    z = 1 - 2 * u
    r = math.sqrt(max(0.0, 1 - z * z))
    om = np.array([r * math.cos(2 * math.pi * v), r * math.sin(2 * math.pi * v), z])
    kap = p["lobe_kappa"][l]
    return 4 * math.pi * kap / (2 * math.pi * (1 - math.exp(-2 * kap))) * math.exp(kap * (om @ p["lobe_dirs"][l] - 1))


def test_pixel_truth_sums_to_total(wl):
    """The per-pixel truths add up to int g = b + w1 int tA h1 + w2 + w3,
    with int tA h1 by an independent fine Gauss-Legendre rule."""
    img = truth.pss_pixel_truth(wl.with_(image=(64, 64)), gl_order=6)
    p = wl.params
    k = 1500
    gx, gw = np.polynomial.legendre.leggauss(k)
    u, w = (gx + 1) / 2, gw / 2
    U, V = np.meshgrid(u, u, indexing="ij")
    ta = 1 + (p["tex_a_amp"][None, None, :] * np.sin(2 * math.pi * (p["tex_a_freq"][:, 0] * U[..., None]
                                                               + p["tex_a_freq"][:, 1] * V[..., None])
                                                + p["tex_a_phase"])).sum(-1) / 8
    z = 1 - 2 * U
    r = np.sqrt(np.maximum(0, 1 - z * z))
    d = p["lobe_dirs"][0]
    kap = p["lobe_kappa"][0]
    dot = d[0] * r * np.cos(2 * math.pi * V) + d[1] * r * np.sin(2 * math.pi * V) + d[2] * z
    h1 = 4 * math.pi * kap / (2 * math.pi * (1 - math.exp(-2 * kap))) * np.exp(kap * (dot - 1))
    w1 = p["lobe_weights"][0]
    total = p["base"][0] + p["lobe_weights"][1] + p["lobe_weights"][2] + w1 * (ta * h1 * np.outer(w, w)).sum()
    assert abs(img.sum() / total - 1) < 1e-5


def test_whole_run_image_matches_truth_by_tiles(oracle_lib, wl):
    """Restore image estimate (c_tilde / j) sum dt 1_pixel against the
    per-pixel truth, aggregated to 8x8 tiles, with the spread of 8
    independent replicate runs as the error scale."""
    small = wl.with_(image=(64, 64), n_chains=2048, n_steps=150)
    tr = truth.pss_pixel_truth(small, gl_order=6)
    tiles = lambda im: im.reshape(8, 8, 8, 8).sum(axis=(1, 3))
    reps = []
    for r in range(8):
        res = O.run(O.Problem(small, seed=700 + r), 0, small.n_chains)
        reps.append(tiles(O.image_estimate(res)))
    reps = np.array(reps)
    mean, sd = reps.mean(0), reps.std(0, ddof=1) / math.sqrt(len(reps))
    z = (mean - tiles(tr)) / sd
    assert np.abs(z).max() < 5.0
    est = O.estimate(res)
    assert abs(est["p_lambda"] / tr.sum() - 1) < 4 * est["p_lambda_se"] / tr.sum()


def test_batch_ranges_follow_the_floor_rule():
    from oracle import oracle as O
    for n, B in ((10, 3), (16, 16), (17, 4), (1000, 7), (5, 1)):
        ranges = O.batch_ranges(n, B)
        for b, (lo, hi) in enumerate(ranges):
            assert list(range(lo, hi)) == [c for c in range(n) if c * B // n == b]


def test_batch_image_standard_error_is_calibrated():
    """Over independent replicates with a known tour distribution, the
    batch-means standard error of the pixel ratio estimate matches the
    spread of the estimate (mean of se^2 / variance within 10%), and the
    estimate is the pooled ratio c_tilde sum S / sum N."""
    from oracle import oracle as O
    rng = np.random.default_rng(21)
    B, reps, c_tilde = 16, 4000, 3.0
    est, se2 = [], []
    for _ in range(reps):
        tours = 1 + rng.poisson(30, size=B)
        imgs = np.zeros((B, 2, 2))
        for b in range(B):
            y = rng.exponential(2.0, size=(tours[b], 2, 2)) * (rng.uniform(size=(tours[b], 2, 2)) < 0.3)
            imgs[b] = y.sum(axis=0)
        m, s = O.image_batch_estimate(imgs, tours, c_tilde)
        np.testing.assert_allclose(m, c_tilde * imgs.sum(axis=0) / tours.sum(), rtol=1e-14)
        est.append(m[0, 0])
        se2.append(s[0, 0] ** 2)
    est, se2 = np.array(est), np.array(se2)
    assert abs(est.mean() / (c_tilde * 0.6) - 1) < 0.01
    ratio = se2.mean() / est.var()
    assert 0.9 < ratio < 1.1, ratio
    m, s = O.image_batch_estimate(np.ones((1, 3, 3)), np.array([5.0]), 2.0)
    assert np.all(np.isnan(s)) and np.allclose(m, 0.4)
