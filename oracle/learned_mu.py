"""FP64 oracle of the learned regeneration distribution -- TEST
INFRASTRUCTURE ONLY (tests and the benchmark's CPU leg; never the product).

mu_theta = (1 - beta) GMM(MLP_theta(c)) + beta Uniform([0,1]^d), with the
MLP  out = W3 gelu(W2 gelu(W1 c + b1) + b2) + b3  (exact erf GELU) and the
mixture read from out = [logits K | means K*d | log_std K*d].  The training
objective is the time-weighted negative log-likelihood of restore samples,
L = -sum_i w_i log u_theta(x_i) / sum_i w_i: the pairs (x_{i-1}, dt_i) of a
Jump Restore run are time-weighted draws of pi (Sec. 7.4, eq. (approx)).

Everything is plain numpy in float64: the loss from its definition, its
gradient with respect to the mixture outputs from the chain rule written
out, and the MLP backward pass by hand.  Pinned by central finite
differences in the tests.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf, logsumexp


def param_layout(in_dim: int, hidden: int, K: int, d: int):
    O = K * (1 + 2 * d)
    sizes = [("W1", (hidden, in_dim)), ("b1", (hidden,)), ("W2", (hidden, hidden)), ("b2", (hidden,)),
             ("W3", (O, hidden)), ("b3", (O,))]
    out, off = {}, 0
    for name, shp in sizes:
        n = int(np.prod(shp))
        out[name] = (off, shp)
        off += n
    return out, off


def unpack(theta, layout):
    return {k: np.asarray(theta[o:o + int(np.prod(s))], dtype=np.float64).reshape(s) for k, (o, s) in layout.items()}


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def mlp_forward(theta, ctx, in_dim, hidden, K, d):
    layout, _ = param_layout(in_dim, hidden, K, d)
    P = unpack(theta, layout)
    c = np.asarray(ctx, dtype=np.float64).reshape(-1, in_dim)
    z1 = c @ P["W1"].T + P["b1"]
    h1 = gelu(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = gelu(z2)
    out = h2 @ P["W3"].T + P["b3"]
    return out, {"c": c, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "P": P, "layout": layout}


def mlp_backward(cache, dout):
    """Gradient of sum_g dout[g] . out[g] with respect to theta."""
    P, layout = cache["P"], cache["layout"]
    dout = np.asarray(dout, dtype=np.float64).reshape(cache["h2"].shape[0], -1)
    g = {}
    g["W3"] = dout.T @ cache["h2"]
    g["b3"] = dout.sum(0)
    dh2 = dout @ P["W3"]
    dz2 = dh2 * gelu_grad(cache["z2"])
    g["W2"] = dz2.T @ cache["h1"]
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ P["W2"]
    dz1 = dh1 * gelu_grad(cache["z1"])
    g["W1"] = dz1.T @ cache["c"]
    g["b1"] = dz1.sum(0)
    flat = np.zeros(sum(int(np.prod(s)) for _, s in layout.values()))
    for k, (o, s) in layout.items():
        flat[o:o + int(np.prod(s))] = g[k].ravel()
    return flat


def split_gmm(out_row, K, d):
    out_row = np.asarray(out_row, dtype=np.float64)
    return out_row[:K], out_row[K:K + K * d].reshape(K, d), out_row[K + K * d:].reshape(K, d)


def log_u(out_row, x, beta, K, d):
    """log of beta 1_box(x) + (1 - beta) sum_k pi_k N(x; m_k, diag s_k^2)."""
    logits, m, ls = split_gmm(out_row, K, d)
    x = np.asarray(x, dtype=np.float64).reshape(-1, d)
    log_pi = logits - logsumexp(logits)
    z = (x[:, None, :] - m[None]) / np.exp(ls)[None]
    comp = (np.log1p(-beta) + log_pi[None] - 0.5 * d * math.log(2 * math.pi) - ls.sum(1)[None]
            - 0.5 * (z * z).sum(-1))
    inbox = np.all((x >= 0) & (x <= 1), axis=1)
    unif = np.where(inbox, math.log(beta) if beta > 0 else -np.inf, -np.inf)
    return logsumexp(np.concatenate([comp, unif[:, None]], axis=1), axis=1), comp


def nll(out_row, x, w, beta, K, d):
    lu, _ = log_u(out_row, x, beta, K, d)
    w = np.asarray(w, dtype=np.float64)
    return float(-(w * lu).sum() / w.sum())


def nll_grad(out_row, x, w, beta, K, d):
    """dL/d out_row by the chain rule: with r_ik = (1 - beta) pi_k N_k(x_i) /
    u(x_i) and z = (x - m)/s,
      dL/dlogit_k  = -sum_i w_i (r_ik - pi_k sum_j r_ij) / W
      dL/dm_kd     = -sum_i w_i r_ik z_ikd / s_kd / W
      dL/dlog s_kd = -sum_i w_i r_ik (z_ikd^2 - 1) / W."""
    logits, m, ls = split_gmm(out_row, K, d)
    x = np.asarray(x, dtype=np.float64).reshape(-1, d)
    w = np.asarray(w, dtype=np.float64)
    W = w.sum()
    lu, comp = log_u(out_row, x, beta, K, d)
    r = np.exp(comp - lu[:, None])
    pi = np.exp(logits - logsumexp(logits))
    s = np.exp(ls)
    z = (x[:, None, :] - m[None]) / s[None]
    wr = w[:, None] * r
    g_logit = -(wr.sum(0) - pi * wr.sum()) / W
    g_m = -(wr[:, :, None] * z).sum(0) / s / W
    g_ls = -(wr[:, :, None] * (z * z - 1.0)).sum(0) / W
    return np.concatenate([g_logit, g_m.ravel(), g_ls.ravel()])
