"""Exact samplers and closed-form cell probabilities used by the statistical
pins (test infrastructure; no part of either implementation)."""
import math

import numpy as np
from scipy import special


def sample_pi_iso(wl, n, rng):
    """Exact draws from pi = p / p_lambda for an isotropic mixture truncated
    to the unit box: pick a component, draw the Gaussian, reject outside."""
    w = np.asarray(wl.params["weights"])
    m = np.asarray(wl.params["means"])
    s = np.asarray(wl.params["sigmas"])
    out = np.empty((0, wl.d))
    while out.shape[0] < n:
        k = rng.choice(w.shape[0], size=2 * n, p=w / w.sum())
        x = m[k] + s[k][:, None] * rng.standard_normal((2 * n, wl.d))
        x = x[np.all((x >= 0) & (x <= 1), axis=1)]
        out = np.concatenate([out, x])
    return out[:n]


def _phi(z):
    return 0.5 * (1 + special.erf(z / math.sqrt(2)))


def iso_cell_masses(wl, edges):
    """int over every cell of the grid edges x edges (per dimension, d <= 2)
    of the mixture p, in closed form."""
    w = np.asarray(wl.params["weights"])
    m = np.asarray(wl.params["means"])
    s = np.asarray(wl.params["sigmas"])
    lo, hi = edges[:-1], edges[1:]
    total = 0.0
    for k in range(w.shape[0]):
        per_dim = [(_phi((hi - m[k, i]) / s[k]) - _phi((lo - m[k, i]) / s[k])) for i in range(wl.d)]
        if wl.d == 1:
            total = total + w[k] * per_dim[0]
        else:
            total = total + w[k] * np.outer(per_dim[0], per_dim[1])
    return total


def hist2d(x, edges):
    h, _, _ = np.histogram2d(x[:, 0], x[:, 1], bins=[edges, edges])
    return h


def chi2_pvalue(obs, expected_counts, min_expected=5.0):
    """Pearson chi-square p-value with every cell of expected count below
    ``min_expected`` pooled into one cell."""
    from scipy import stats
    obs = np.asarray(obs, dtype=np.float64).ravel()
    e = np.asarray(expected_counts, dtype=np.float64).ravel()
    small = e < min_expected
    o2 = np.concatenate([obs[~small], [obs[small].sum()]])
    e2 = np.concatenate([e[~small], [e[small].sum()]])
    if e2[-1] == 0:
        if o2[-1] > 0:
            return 0.0
        o2, e2 = o2[:-1], e2[:-1]
    e2 = e2 * o2.sum() / e2.sum()
    return float(stats.chisquare(o2, e2).pvalue)


def mixture_mu_from_target(wl, beta=0.1):
    """A diagonal-Gaussian-mixture mu built from a full-covariance target's
    own weights, means and marginal variances, with a defensive uniform
    share beta (the shape of the learned regeneration distribution)."""
    c = wl.params["covs"]
    return {"logits": np.log(wl.params["weights"]), "means": wl.params["means"],
            "log_std": 0.5 * np.log(np.stack([np.diag(ci) for ci in c])), "beta": beta}
