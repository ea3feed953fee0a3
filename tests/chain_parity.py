"""Shared bookkeeping of the GPU parity tests (test infrastructure; no part
of either implementation).

Where the float32 HIP path and the float64 oracle may legitimately decide
differently: a decision compares two log quantities, and its margin (the
oracle's ln t2 - ln t1 for a kill, ln u - ln alpha for an accept) can be
smaller than the float32 error of the log densities that enter it.  Those
errors are relative to the size of the log densities (the exponent terms of
a mixture component are evaluated to a few float32 ulps of themselves), so
a margin is scaled by 1 + the sum of the magnitudes of the log densities it
compares, and a decision is a near-tie when the scaled margin is below
TAU = 1e-5 -- the blueprint's near-tie margin, per unit of log density.  A
category pick of a learned-form mu is a near-tie when its uniform lies
within TAU_CAT of a cumulative-weight boundary (the boundaries are float32
on the GPU).  A small-step proposal is a near-tie when it lies within
(moves + 1) 2^-21 of the edge of the chain's support (the box, or its tile):
the float32 state differs from the oracle's by at most one rounding (2^-24
relative, plus the float32 error of the step itself) per local move since
it was last drawn exactly from mu, so it may land on the other side.  A
chain whose trajectory saw no near-tie must reproduce the
oracle's tour count exactly and its tour sums within the float32 bounds
below; a chain that saw one may diverge from that step on and is excluded
(and counted).

Float32 bounds, with eps = 1e-5 (1 + L) the relative error of one holding
time or one value of p (L bounds |log p| + |log u| where the time mass is,
i.e. at the largest densities; 4e-5 more for the 12-D integrand, whose
kappa = 1e3 lobes amplify the rounding of the direction):
  * tour time: n float32 additions per chain and eps per term,
    |T_gpu - T| <= (n 2^-24 + eps) T;
  * tour integral of f = p: one eps more for p;
  * terms below float32's smallest normal number 2^-126 are flushed on the
    GPU (8-D regenerations far from the modes have p dt ~ 1e-40): 2^-126 per
    step of absolute error on top;
  * these bounds count the rounding of each term, not the growth of a state
    difference along a long run of local moves: a MALA proposal carries
    (eps^2 / 2) grad log p, whose Hessian (up to 1 / 1e-4 in the 8-D
    mixture) can amplify it by ~1.1 per move, so whole runs are compared
    chain by chain where tours are short or moves are random walks (the 2-D
    and image workloads, the 8-D workloads at their provable c~) and by
    their estimates elsewhere;
  * an image pixel: two orders of n positive float32 additions differ by at
    most 2 (n + 1) 2^-24 of the sum (n splats in the pixel), plus eps, plus
    the dt of every splat whose state lies so close to a pixel edge that the
    float32 state, which differs from the oracle's by the rounding of the
    local moves since the last regeneration, may fall on the other side (the
    oracle's image_near).
"""
from __future__ import annotations

import numpy as np

TAU = 1e-5
TAU_CAT = 1e-6
EDGE = 2.0 ** -21   # per local move since the last regeneration


def scaled_step_margins(margins: np.ndarray):
    """Scaled kill and accept margins of single transitions, from the
    margins array of oracle.transitions (inf where no such decision was
    made or a log density is infinite: no tie is possible there)."""
    m = np.asarray(margins, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        sx = 1.0 + np.abs(m[:, 5]) + np.abs(m[:, 6])
        kill = np.abs(m[:, 0]) / sx
        sy = sx + np.abs(m[:, 3]) + np.abs(m[:, 4])
        acc = np.abs(m[:, 1]) / sy
    kill = np.where(np.isfinite(kill), kill, np.inf)
    acc = np.where(np.isfinite(acc), acc, np.inf)
    # a proposal at the edge of the support: accepted on one side, outside
    # (p = 0, rejected) on the other
    acc = np.where(m[:, 7] < EDGE, 0.0, acc)
    return kill, acc


def near_tie_chains(min_margin: np.ndarray) -> np.ndarray:
    mm = np.asarray(min_margin)
    return (mm[:, 0] < TAU) | (mm[:, 1] < TAU) | (mm[:, 2] < TAU_CAT) | (mm[:, 3] < EDGE)


def log_scale(wl, mu=None) -> float:
    """L: a bound of |log p| + |log u| at the states that carry the time
    mass (the largest densities): ln of the peak bound of p, plus ln of the
    peak of a mixture mu."""
    from oracle import choose_c_tilde
    L = abs(np.log(choose_c_tilde.peak_bound(wl)))
    if mu is not None:
        ls = np.asarray(mu["log_std"], dtype=np.float64).reshape(len(np.asarray(mu["logits"]).ravel()), -1)
        d = ls.shape[1]
        L += float(np.max(np.abs(-0.5 * d * np.log(2 * np.pi) - ls.sum(axis=1))))
    return float(L)


def eps_dt(wl, mu=None) -> float:
    return 1e-5 * (1.0 + log_scale(wl, mu)) + (4e-5 if wl.target == "pss" else 0.0)


def check_chain_sums(gpu: dict, ores, wl, mu=None, say=print, label: str = "") -> dict:
    """Every chain without a near-tie: identical tour count, tour time and
    tour integral within the float32 bounds.  gpu holds n_done, t_done and
    optionally a_done for the same chains as ores (in order).  Returns the
    near-tie mask and the mismatch mask (mismatches are allowed only at
    near-tie chains)."""
    near = near_tie_chains(ores.min_margin)
    n_g = np.asarray(gpu["n_done"]).astype(np.int64)
    same_n = n_g == ores.n_done
    eps = eps_dt(wl, mu)
    n_tr = np.asarray(ores.transitions, dtype=np.float64)
    rel_t = n_tr * 2.0 ** -24 + eps
    t_g, t_o = np.asarray(gpu["t_done"], dtype=np.float64), ores.t_done
    err_t = np.abs(t_g - t_o) / np.maximum(np.abs(t_o), 1e-300)
    # terms below float32's smallest normal number (2^-126) are lost on the
    # GPU: one such unit per step on top of the relative bound
    tiny = n_tr * 2.0 ** -126
    err_t = np.where(np.abs(t_g - t_o) <= tiny, 0.0, err_t)
    ok = same_n & ((err_t <= rel_t) | (t_g == t_o))
    ratio_t = np.where(t_o != 0, err_t / rel_t, 0.0)
    ratio_a = np.zeros_like(ratio_t)
    if "a_done" in gpu and gpu["a_done"] is not None:
        a_g, a_o = np.asarray(gpu["a_done"], dtype=np.float64), ores.a_done
        rel_a = rel_t + eps
        err_a = np.abs(a_g - a_o) / np.maximum(np.abs(a_o), 1e-300)
        err_a = np.where(np.abs(a_g - a_o) <= tiny, 0.0, err_a)
        ok &= (err_a <= rel_a) | (a_g == a_o)
        ratio_a = np.where(a_o != 0, err_a / rel_a, 0.0)
    clean = ~near
    mism = ~ok
    say(f"[{label}] chains {len(n_g)}: near-tie {int(near.sum())}, mismatched {int(mism.sum())} "
        f"(all near-tie: {bool(np.all(near[mism]))}); clean chains: max err/bound tour time "
        f"{float(ratio_t[clean].max()) if clean.any() else 0:.3f}, tour integral "
        f"{float(ratio_a[clean].max()) if clean.any() else 0:.3f}")
    assert not np.any(mism & clean), f"{int(np.sum(mism & clean))} chains without a near-tie differ from the oracle"
    return {"near": near, "mismatch": mism}


def clean_ranges(near: np.ndarray, c0: int = 0):
    """Maximal ranges [lo, hi) of consecutive chains without a near-tie
    (chain ids offset by c0)."""
    out, lo = [], None
    for i, bad in enumerate(np.asarray(near)):
        if not bad and lo is None:
            lo = i
        if bad and lo is not None:
            out.append((c0 + lo, c0 + i))
            lo = None
    if lo is not None:
        out.append((c0 + lo, c0 + len(near)))
    return out


def check_image(img_gpu: np.ndarray, img_o: np.ndarray, count: np.ndarray, near: np.ndarray, eps: float,
                say=print, label: str = "") -> float:
    """Pixel-by-pixel parity of an image of float32 splat sums with the
    oracle's float64 sums over the same chains; returns max err / bound."""
    g = np.asarray(img_gpu, dtype=np.float64)
    o = np.asarray(img_o, dtype=np.float64)
    bound = o * (2.0 * (np.asarray(count) + 1.0) * 2.0 ** -24 + eps) + np.asarray(near) + 1e-30
    err = np.abs(g - o)
    r = float((err / bound).max())
    say(f"[{label}] pixels {o.size}: nonzero {int((o > 0).sum())}, max err/bound {r:.3f}, max rel err "
        f"{float((err / np.maximum(o, 1e-300))[o > 0].max()) if (o > 0).any() else 0:.2e}, "
        f"edge mass {float(np.asarray(near).sum() / 9 / max(o.sum(), 1e-300)):.2e} of the image")
    assert np.all(err <= bound), f"{int((err > bound).sum())} pixels outside the float32 bound"
    return r
