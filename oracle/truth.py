"""Closed-form and library truths for the synthetic targets -- test
infrastructure only.

These are the quantities the restore estimates converge to:

* p_lambda   = int_box p dlambda                     (Sec. 4, eq. (targetdensity-assumption-1))
* lam_pf     = lambda(p f) with f = p, i.e. int_box p^2
* pi_f       = lam_pf / p_lambda

For isotropic mixtures everything is a product of one-dimensional Gaussian
box probabilities (erf), using the identity that a product of Gaussian
densities is a scaled Gaussian density.  For full-covariance mixtures the
box probabilities come from scipy's multivariate normal CDF (Genz's
quasi-Monte Carlo), a library routine, so those truths carry a small
integration error of their own.
"""
from __future__ import annotations

import itertools
import math
from typing import Sequence

import numpy as np
from scipy import special, stats


def _box_prob_1d(m, s):
    """P(0 <= X <= 1) for X ~ N(m, s^2), elementwise."""
    m = np.asarray(m, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    return 0.5 * (special.erf((1.0 - m) / (s * math.sqrt(2.0))) + special.erf(m / (s * math.sqrt(2.0))))


def iso_product_box_integral(means: Sequence[np.ndarray], sigmas: Sequence[float]) -> float:
    """int_{[0,1]^d} prod_i N(x; m_i, s_i^2 I) dx, for any number of factors.

    Per dimension, prod_i N(x; m_i, s_i^2) = G * N(x; m_c, s_c^2) with
    1/s_c^2 = sum 1/s_i^2, m_c = s_c^2 sum m_i/s_i^2 and
    G = sqrt(2 pi s_c^2) / prod sqrt(2 pi s_i^2) * exp(-R/2),
    R = sum m_i^2/s_i^2 - m_c^2/s_c^2."""
    means = [np.asarray(m, dtype=np.float64) for m in means]
    sig = np.asarray(sigmas, dtype=np.float64)
    prec = 1.0 / (sig * sig)
    pc = prec.sum()
    sc2 = 1.0 / pc
    total = 1.0
    for dim in range(means[0].shape[0]):
        md = np.array([m[dim] for m in means])
        mc = sc2 * (md * prec).sum()
        R = (md * md * prec).sum() - mc * mc * pc
        G = math.sqrt(2 * math.pi * sc2) / np.prod(np.sqrt(2 * math.pi * sig * sig)) * math.exp(-0.5 * R)
        total *= G * float(_box_prob_1d(mc, math.sqrt(sc2)))
    return total


def gmm_iso_power_integral(wl, power: int) -> float:
    """int_box p^power for an isotropic mixture p (power 1: p_lambda)."""
    w = np.asarray(wl.params["weights"], dtype=np.float64)
    m = np.asarray(wl.params["means"], dtype=np.float64)
    s = np.asarray(wl.params["sigmas"], dtype=np.float64)
    K = w.shape[0]
    total = 0.0
    for combo in itertools.product(range(K), repeat=power):
        coef = float(np.prod(w[list(combo)]))
        total += coef * iso_product_box_integral([m[k] for k in combo], [s[k] for k in combo])
    return total


def _mvn_box_prob(mean, cov) -> float:
    d = mean.shape[0]
    if d == 1:
        return float(_box_prob_1d(mean[0], math.sqrt(cov[0, 0])))
    # Genz's randomised lattice rule keeps its own generator state between
    # calls, so a value depends on the calls before it within its error
    # (observed ~3e-7 here): reproducible to that accuracy, not bit for bit.
    return float(stats.multivariate_normal.cdf(np.ones(d), mean=mean, cov=cov, maxpts=200000 * d,
                                               abseps=1e-9, releps=1e-7, lower_limit=np.zeros(d)))


def gmm_full_p_lambda(wl) -> float:
    w = np.asarray(wl.params["weights"])
    m = np.asarray(wl.params["means"])
    c = np.asarray(wl.params["covs"])
    return float(sum(w[k] * _mvn_box_prob(m[k], c[k]) for k in range(w.shape[0])))


def gmm_full_p2(wl) -> float:
    """int_box p^2 = sum_ab w_a w_b N(m_a; m_b, S_a + S_b) P_box(N(m_c, S_c)),
    S_c = (S_a^-1 + S_b^-1)^-1, m_c = S_c (S_a^-1 m_a + S_b^-1 m_b)."""
    w = np.asarray(wl.params["weights"])
    m = np.asarray(wl.params["means"])
    c = np.asarray(wl.params["covs"])
    K = w.shape[0]
    P = np.linalg.inv(c)
    total = 0.0
    for a in range(K):
        for b in range(K):
            Sc = np.linalg.inv(P[a] + P[b])
            Sc = 0.5 * (Sc + Sc.T)
            mc = Sc @ (P[a] @ m[a] + P[b] @ m[b])
            G = stats.multivariate_normal(mean=m[b], cov=c[a] + c[b]).pdf(m[a])
            total += w[a] * w[b] * G * _mvn_box_prob(mc, Sc)
    return float(total)


def truths(wl) -> dict:
    """p_lambda, lam_pf (f = p) and pi_f of a mixture workload."""
    if wl.target == "gmm_iso":
        pl = gmm_iso_power_integral(wl, 1)
        p2 = gmm_iso_power_integral(wl, 2)
    elif wl.target == "gmm_full":
        pl = gmm_full_p_lambda(wl)
        p2 = gmm_full_p2(wl)
    else:
        raise ValueError(wl.target)
    return {"p_lambda": pl, "lam_pf": p2, "pi_f": p2 / pl}


# ---------------------------------------------------------------------------
# rendering-shaped integrand: per-pixel truth
# ---------------------------------------------------------------------------

def _texture_pixel_integral(freq, amp, phase, x0, x1, y0, y1):
    """int over [x0,x1]x[y0,y1] of t(y) = 1 + (1/8) sum a_m sin(2 pi n.y + phi)
    in closed form (nested antiderivatives of the sine)."""
    val = (x1 - x0) * (y1 - y0)
    for m in range(freq.shape[0]):
        a, b = 2 * math.pi * freq[m, 0], 2 * math.pi * freq[m, 1]
        ph = phase[m]

        def F(u, v):
            # antiderivative of sin(a u + b v + ph) in u then v
            if a != 0 and b != 0:
                return -np.sin(a * u + b * v + ph) / (a * b)
            if a != 0:  # b == 0: int_v is v * (-cos(a u + ph)/a)
                return -v * np.cos(a * u + ph) / a
            return -u * np.cos(b * v + ph) / b  # a == 0, b != 0

        s = F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0)
        val = val + amp[m] * s / 8.0
    return val


def pss_pixel_truth(wl, gl_order: int = 8) -> np.ndarray:
    """lambda(g 1_pixel) for every pixel of the rendering-shaped integrand.

    Integrating out x2..x11 (tB and lobes 2, 3 each integrate to 1) leaves
    tA(x0,x1) (b + w2 + w3 + w1 h1(x0,x1)); the first part is closed form,
    the lobe part uses gl_order x gl_order Gauss-Legendre per pixel."""
    W, H = wl.image
    p = wl.params
    fa, aa, pa = p["tex_a_freq"], p["tex_a_amp"], p["tex_a_phase"]
    wts = p["lobe_weights"]
    base = float(p["base"][0]) + float(wts[1]) + float(wts[2])
    xs = np.arange(W + 1) / W
    ys = np.arange(H + 1) / H
    X0, Y0 = np.meshgrid(xs[:-1], ys[:-1])
    X1, Y1 = np.meshgrid(xs[1:], ys[1:])
    img = base * _texture_pixel_integral(fa, aa, pa, X0, X1, Y0, Y1)
    # lobe 1 on (x0, x1)
    g, gw = np.polynomial.legendre.leggauss(gl_order)
    dirv = p["lobe_dirs"][0]
    kappa = float(p["lobe_kappa"][0])
    acc = np.zeros((H, W))
    for i in range(gl_order):
        for j in range(gl_order):
            u = X0 + (g[i] + 1) * 0.5 / W
            v = Y0 + (g[j] + 1) * 0.5 / H
            z = 1 - 2 * u
            r = np.sqrt(np.maximum(0, 1 - z * z))
            dot = dirv[0] * r * np.cos(2 * math.pi * v) + dirv[1] * r * np.sin(2 * math.pi * v) + dirv[2] * z
            h = 4 * math.pi * kappa / (2 * math.pi * (1 - math.exp(-2 * kappa))) * np.exp(kappa * (dot - 1))
            ta = 1 + (aa[None, None, :] * np.sin(2 * math.pi * (fa[:, 0][None, None, :] * u[..., None]
                                                                  + fa[:, 1][None, None, :] * v[..., None])
                                                  + pa[None, None, :])).sum(-1) / 8
            acc += gw[i] * gw[j] * ta * h
    img = img + float(wts[0]) * acc * 0.25 / (W * H)
    return img
