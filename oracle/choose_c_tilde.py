"""The killing-rate constant used for the mixture workloads.

Any c_tilde > 0 gives a pi-invariant restore process (the killing rate of
the simplified form needs only pi-invariant local dynamics).  The step
budget B and the drain cap make long tours costly and, if they outlive the
cap, censored.  The rule used here bounds the expected lifetime
p(x) / (c_tilde u(x)) by B/8 at every x of the box:

    c_tilde = max(1, 8 P / B),   P = sum_k w_k (2 pi)^(-d/2) det(S_k)^(-1/2),

where P >= sup p because every component density is at most its peak value.
Run as a script to print the constant stored in ``workloads``.
"""
import math
import sys

import numpy as np


def peak_bound(wl) -> float:
    if wl.target == "pss":
        # g <= max tA * max tB * (b + sum_l w_l max h_l), max t <= 1 + sum |a_m| / 8,
        # max h = 4 pi kappa / (2 pi (1 - e^{-2 kappa}))
        p = wl.params
        ta = 1 + np.abs(p["tex_a_amp"]).sum() / 8
        tb = 1 + np.abs(p["tex_b_amp"]).sum() / 8
        k = np.asarray(p["lobe_kappa"], dtype=np.float64)
        hmax = 2 * k / -np.expm1(-2 * k)
        return float(ta * tb * (p["base"][0] + (np.asarray(p["lobe_weights"]) * hmax).sum()))
    w = np.asarray(wl.params["weights"], dtype=np.float64)
    d = wl.d
    if wl.target == "gmm_iso":
        s = np.asarray(wl.params["sigmas"], dtype=np.float64)
        return float((w * (2 * math.pi * s * s) ** (-d / 2)).sum())
    c = np.asarray(wl.params["covs"], dtype=np.float64)
    return float((w * (2 * math.pi) ** (-d / 2) / np.sqrt(np.linalg.det(c))).sum())


def c_tilde_rule(wl, sig: int = 3) -> float:
    v = max(1.0, 8.0 * peak_bound(wl) / wl.n_steps)
    return float(f"{v:.{sig - 1}e}")


def c_tilde_unadjusted(wl, grid: int = 201, sig: int = 2) -> float:
    """Local dynamics that are not pi-invariant (the unadjusted random-walk
    jump process) need k = (c_tilde u + Q^T p - p) / p >= 0 everywhere
    (Sec. 6.2, eq. (killing-rate)), i.e. c_tilde >= sup_box (p - Q^T p) / u
    with u = 1 (uniform mu).  The supremum is located on a grid over the box
    (oracle densities), refined by Nelder-Mead from the best grid point,
    and doubled for margin; the result is rounded up."""
    from scipy.optimize import minimize
    from oracle import oracle as O
    prob = O.Problem(wl)

    def excess(x):
        x = np.clip(np.asarray(x, dtype=np.float64).reshape(-1, wl.d), 0.0, 1.0)
        return np.exp(O.log_target(prob, x)) - np.exp(O.log_inflow(prob, x))

    g = np.linspace(0.0, 1.0, grid)
    X = np.stack(np.meshgrid(*([g] * wl.d), indexing="ij"), axis=-1).reshape(-1, wl.d)
    e = excess(X)
    best = minimize(lambda x: -excess(x)[0], X[np.argmax(e)], method="Nelder-Mead",
                    options={"xatol": 1e-7, "fatol": 1e-10})
    sup = max(float(e.max()), -float(best.fun))
    v = 2.0 * sup
    scale = 10.0 ** (math.floor(math.log10(v)) - (sig - 1))
    return math.ceil(v / scale) * scale


if __name__ == "__main__":
    sys.path.insert(0, __file__.rsplit("/oracle/", 1)[0])
    from workloads import gmm_full, gmm_iso_2d, pss_render
    print("gmm_iso_2d", c_tilde_rule(gmm_iso_2d()))
    print("gmm_full_8d", c_tilde_rule(gmm_full()))
    print("pss_render_12d", c_tilde_rule(pss_render()))
    print("gmm_iso_2d with the unadjusted random-walk jump process",
          c_tilde_unadjusted(gmm_iso_2d().with_(local="rw_unadjusted", c_tilde=1.0)))
