"""Pins of the FP64 learned-mu oracle: its analytic gradients against
central finite differences of its loss, and its mixture density against
the C oracle's mu density (two independent writings) and normalisation."""
import math

import numpy as np

from oracle import learned_mu as L
from oracle import oracle as O


def _setup(seed=0, K=5, d=3, in_dim=4, H=6, G=2):
    rng = np.random.default_rng(seed)
    _, n = L.param_layout(in_dim, H, K, d)
    theta = 0.3 * rng.standard_normal(n)
    ctx = rng.standard_normal((G, in_dim))
    x = rng.uniform(-0.1, 1.1, size=(200, d))
    w = rng.exponential(size=200)
    return rng, theta, ctx, x, w, K, d, in_dim, H


def test_nll_gradient_matches_finite_differences():
    rng, theta, ctx, x, w, K, d, in_dim, H = _setup()
    out, _ = L.mlp_forward(theta, ctx, in_dim, H, K, d)
    row = out[0]
    g = L.nll_grad(row, x, w, 0.1, K, d)
    h = 1e-6
    for j in range(row.size):
        e = np.zeros_like(row)
        e[j] = h
        fd = (L.nll(row + e, x, w, 0.1, K, d) - L.nll(row - e, x, w, 0.1, K, d)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), j


def test_mlp_backward_matches_finite_differences():
    rng, theta, ctx, x, w, K, d, in_dim, H = _setup(seed=1)
    out, cache = L.mlp_forward(theta, ctx, in_dim, H, K, d)
    dout = rng.standard_normal(out.shape)
    g = L.mlp_backward(cache, dout)
    f = lambda th: float((L.mlp_forward(th, ctx, in_dim, H, K, d)[0] * dout).sum())
    h = 1e-6
    for j in rng.choice(theta.size, 60, replace=False):
        e = np.zeros_like(theta)
        e[j] = h
        fd = (f(theta + e) - f(theta - e)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), j


def test_chain_rule_through_mlp_and_nll():
    rng, theta, ctx, x, w, K, d, in_dim, H = _setup(seed=2, G=1)
    out, cache = L.mlp_forward(theta, ctx, in_dim, H, K, d)
    g = L.mlp_backward(cache, L.nll_grad(out[0], x, w, 0.2, K, d)[None])
    f = lambda th: L.nll(L.mlp_forward(th, ctx, in_dim, H, K, d)[0][0], x, w, 0.2, K, d)
    h = 1e-6
    for j in rng.choice(theta.size, 40, replace=False):
        e = np.zeros_like(theta)
        e[j] = h
        fd = (f(theta + e) - f(theta - e)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), j


def test_mixture_density_matches_c_oracle(oracle_lib):
    from workloads import gmm_full
    rng = np.random.default_rng(3)
    K, d = 7, 8
    row = np.concatenate([rng.standard_normal(K), rng.uniform(0.2, 0.8, K * d), np.log(rng.uniform(0.02, 0.2, K * d))])
    logits, m, ls = L.split_gmm(row, K, d)
    wl = gmm_full(n_chains=16)
    prob = O.Problem(wl, mu={"logits": logits, "means": m, "log_std": ls, "beta": 0.15})
    x = np.concatenate([rng.uniform(0, 1, (50, d)), m + 0.05 * rng.standard_normal((K, d)),
                        rng.uniform(-0.2, 1.2, (20, d))])
    lu, _ = L.log_u(row, x, 0.15, K, d)
    np.testing.assert_allclose(lu, O.log_mu(prob, x), rtol=1e-12, atol=1e-12)


def test_mixture_density_integrates_to_one():
    rng = np.random.default_rng(4)
    K, d = 4, 2
    row = np.concatenate([rng.standard_normal(K), rng.uniform(0.3, 0.7, K * d), np.log(rng.uniform(0.05, 0.1, K * d))])
    g, gw = np.polynomial.legendre.leggauss(300)
    lo, hi = -0.5, 1.5
    pts, wq = lo + (hi - lo) * (g + 1) / 2, gw * (hi - lo) / 2
    X, Y = np.meshgrid(pts, pts, indexing="ij")
    lu, _ = L.log_u(row, np.stack([X.ravel(), Y.ravel()], 1), 0.25, K, d)
    inside = ((X >= 0) & (X <= 1) & (Y >= 0) & (Y <= 1)).ravel()
    gauss = np.exp(lu) - 0.25 * inside
    assert abs((gauss.reshape(X.shape) * np.outer(wq, wq)).sum() - 0.75) < 1e-6
