"""Seeded parameter generators for the synthetic restore workloads.

Every workload is a target density p on the unit box [0,1]^d (p = 0
outside), a regeneration distribution mu (uniform on the box unless stated
otherwise), a local Metropolis-Hastings kernel and a chain population.  The
paper measures on rendering scenes that are not available here; these
synthetic targets stand in for them (a 2-D and an 8-D Gaussian mixture, a
12-D primary-sample-space integrand mapped to a 512x512 image, and a batch
of 256 uneven mixtures).

Only numpy's PCG64 generator is used, with the seeds recorded in each
workload, so the oracle and the HIP path receive bit-identical float64
parameters.  Nothing here evaluates a density or any other quantity of the
restore method; the parameters are returned in canonical form (weights,
means, covariances; texture frequencies, amplitudes, phases; lobe
directions) and each side derives its own factorisations.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Workload:
    """One synthetic restore workload.

    Attributes
    ----------
    name:        short identifier.
    target:      "gmm_iso" | "gmm_full" | "pss".
    d:           state dimension.
    K:           number of mixture components (0 for "pss").
    params:      canonical float64 parameters (see each generator).
    local:       "rwmh" (Gaussian random walk) | "mala" (Langevin proposal)
                 | "hmc" (Hamiltonian Monte Carlo, leapfrog) | "rw_unadjusted"
                 (random-walk jumps without acceptance test: not pi-invariant).
    step:        random-walk sigma, MALA epsilon or HMC leapfrog step size.
    n_leapfrog:  leapfrog steps per HMC update (0 for the other kernels).
    tile_px:     image integrand: tile edge of a tile-stratified run (0 off).
    n_chains:    chain population size.
    n_steps:     step budget B (steps with regeneration).
    drain_cap:   extra steps allowed to finish the tour straddling B.
    c_tilde:     the killing-rate constant (k = c_tilde * u / p).
    seed:        chain seed (Philox key).
    problem_seed: seed that drew ``params``.
    image:       (width, height) for the pixel integrand, or None.
    image_batches: contiguous chain ranges with an image each (per-pixel
                 standard errors); 0 or 1 = one image.
    """

    name: str
    target: str
    d: int
    K: int
    params: Dict[str, np.ndarray]
    local: str
    step: float
    n_chains: int
    n_steps: int
    drain_cap: int
    c_tilde: float
    seed: int
    problem_seed: int
    image: Optional[tuple] = None
    image_batches: int = 0
    n_leapfrog: int = 0
    tile_px: int = 0

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# ---------------------------------------------------------------------------
# helpers (parameter drawing only)
# ---------------------------------------------------------------------------

def _haar_rotation(rng: np.random.Generator, d: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    signs of R's diagonal moved into Q (Mezzadri's recipe)."""
    a = rng.standard_normal((d, d))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    return q


def _full_cov_mixture(rng: np.random.Generator, d: int, K: int,
                      eig_lo: float = 1e-4, eig_hi: float = 1e-2,
                      mean_lo: float = 0.2, mean_hi: float = 0.8):
    means = rng.uniform(mean_lo, mean_hi, size=(K, d))
    weights = rng.dirichlet(np.ones(K))
    covs = np.empty((K, d, d))
    for k in range(K):
        rot = _haar_rotation(rng, d)
        eig = np.exp(rng.uniform(math.log(eig_lo), math.log(eig_hi), size=d))
        c = (rot * eig[None, :]) @ rot.T
        covs[k] = 0.5 * (c + c.T)
    return weights, means, covs


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def gmm_iso_2d(n_chains: int = 4096, n_steps: int = 1000,
               problem_seed: int = 1001, seed: int = 2001) -> Workload:
    """2-D target: 4-component isotropic Gaussian mixture, sigma = 0.05,
    weights 0.4/0.3/0.2/0.1, means uniform in [0.2,0.8]^2, restricted to
    [0,1]^2.  Random-walk MH with sigma 0.02, uniform mu, c_tilde = 1."""
    rng = np.random.default_rng(problem_seed)
    means = rng.uniform(0.2, 0.8, size=(4, 2))
    params = {
        "weights": np.array([0.4, 0.3, 0.2, 0.1]),
        "means": means,
        "sigmas": np.full(4, 0.05),
    }
    return Workload("gmm_iso_2d", "gmm_iso", 2, 4, params, "rwmh", 0.02,
                    n_chains, n_steps, 4 * n_steps, 1.0, seed, problem_seed)


# c_tilde of the 2-D workload with the unadjusted random-walk jump process:
# twice sup over the box of (p - Q^T p) / u, so that the killing rate
# (c_tilde u + Q^T p - p) / p stays positive everywhere.  Written by
# oracle/choose_c_tilde.py.
C_TILDE_GMM_ISO_2D_UNADJUSTED = 7.7


def gmm_iso_2d_unadjusted(n_chains: int = 4096, n_steps: int = 1000, problem_seed: int = 1001,
                          seed: int = 2001) -> Workload:
    """The 2-D target with local dynamics that are not pi-invariant: the
    unadjusted random-walk jump process (rate 1, every jump x + sigma z
    taken, sigma 0.02), whose killing rate carries the adjoint generator
    term L* p = Q^T p - p."""
    return gmm_iso_2d(n_chains, n_steps, problem_seed, seed).with_(
        name="gmm_iso_2d_unadjusted", local="rw_unadjusted", c_tilde=C_TILDE_GMM_ISO_2D_UNADJUSTED)


# c_tilde of the 8-D workload: 8 * P / B with P = sum_k w_k (2 pi)^(-d/2)
# det(Sigma_k)^(-1/2), an upper bound of p on the box, so the mean lifetime
# is at most B/8 steps everywhere and tours that outlive the drain cap are
# practically impossible.  Written by oracle/choose_c_tilde.py.
C_TILDE_GMM_FULL_8D = 3.34e7


def gmm_full(d: int = 8, K: int = 16, n_chains: int = 1 << 20,
             n_steps: int = 512, problem_seed: int = 1002, seed: int = 2002,
             local: str = "mala", step: float = 0.005,
             c_tilde: Optional[float] = None) -> Workload:
    """d-D target: K-component full-covariance Gaussian mixture, covariance
    eigenvalues log-uniform in [1e-4, 1e-2] with Haar rotations, means
    uniform in [0.2,0.8]^d, Dirichlet(1) weights, restricted to [0,1]^d.
    MALA with epsilon 0.005 by default, uniform mu."""
    rng = np.random.default_rng(problem_seed)
    w, m, c = _full_cov_mixture(rng, d, K)
    params = {"weights": w, "means": m, "covs": c}
    if c_tilde is None:
        c_tilde = C_TILDE_GMM_FULL_8D if (d, K, problem_seed) == (8, 16, 1002) else 1.0
    return Workload(f"gmm_full_{d}d", "gmm_full", d, K, params, local, step,
                    n_chains, n_steps, 4 * n_steps, float(c_tilde), seed,
                    problem_seed)


# c_tilde of the rendering-shaped workload by the same rule, with the bound
# max tA * max tB * (b + sum_l w_l max h_l) of g.  Written by
# oracle/choose_c_tilde.py.
C_TILDE_PSS_12D = 155.0


def pss_render(n_chains: int = 1 << 20, n_steps: int = 256,
               problem_seed: int = 1003, seed: int = 2003,
               image=(512, 512), c_tilde: float = C_TILDE_PSS_12D,
               image_batches: int = 16) -> Workload:
    """12-D rendering-shaped integrand on [0,1]^12.

    g(x) = tA(x0,x1) * tB(x6..x11) * [b + sum_l w_l h_l(x_{2l-2}, x_{2l-1})]
    with two procedural textures t(y) = 1 + (1/8) sum_m a_m sin(2 pi <n_m,y>
    + phi_m) (8 seeded sinusoids each, integer frequencies n_m != 0,
    |a_m| <= 0.9) and three von Mises-Fisher lobes of concentration kappa
    on the sphere, reached from the unit square by z = 1 - 2u, phi = 2 pi v.
    Coordinates (x0, x1) select the pixel of a width x height image; the
    chains are split into ``image_batches`` ranges with an image each."""
    rng = np.random.default_rng(problem_seed)

    def texture(dim):
        n = np.zeros((8, dim), dtype=np.int64)
        for mrow in range(8):
            while True:
                cand = rng.integers(-3, 4, size=dim)
                if np.any(cand != 0):
                    break
            n[mrow] = cand
        a = rng.uniform(-0.9, 0.9, size=8)
        phi = rng.uniform(0.0, 2 * math.pi, size=8)
        return n.astype(np.float64), a, phi

    nA, aA, pA = texture(2)
    nB, aB, pB = texture(6)
    z = rng.uniform(-0.8, 0.8, size=3)
    ph = rng.uniform(0.0, 2 * math.pi, size=3)
    s = np.sqrt(1 - z * z)
    lobes = np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)
    params = {
        "tex_a_freq": nA, "tex_a_amp": aA, "tex_a_phase": pA,
        "tex_b_freq": nB, "tex_b_amp": aB, "tex_b_phase": pB,
        "lobe_dirs": lobes,
        "lobe_kappa": np.full(3, 1000.0),
        "lobe_weights": np.full(3, 1.0 / 3.0),
        "base": np.array([0.05]),
    }
    return Workload("pss_render_12d", "pss", 12, 0, params, "rwmh", 0.02,
                    n_chains, n_steps, 4 * n_steps, float(c_tilde), seed,
                    problem_seed, image=tuple(image) if image else None,
                    image_batches=int(image_batches) if image else 0)


def batched_uneven(n_targets: int = 256, problem_seed: int = 1005,
                   seed: int = 2005, n_steps: int = 256,
                   chains_lo: int = 1 << 10, chains_hi: int = 1 << 18) -> List[Workload]:
    """256 independent full-covariance mixtures: d uniform in {2..16}, K
    uniform in {2..32}, chain count log-uniform in [2^10, 2^18], all drawn
    from one seeded stream.  Random-walk MH with sigma 0.02, uniform mu.
    Target t uses Philox target id t."""
    rng = np.random.default_rng(problem_seed)
    out = []
    for t in range(n_targets):
        d = int(rng.integers(2, 17))
        K = int(rng.integers(2, 33))
        n_chains = int(round(math.exp(rng.uniform(math.log(chains_lo), math.log(chains_hi)))))
        w, m, c = _full_cov_mixture(rng, d, K)
        # c_tilde by the same lifetime rule as the single workloads (mean
        # lifetime <= B/8 under the peak bound sum_k w_k N_k(m_k; m_k, S_k))
        peak = float((w * (2 * math.pi) ** (-d / 2) / np.sqrt(np.linalg.det(c))).sum())
        c_tilde = float(f"{max(1.0, 8.0 * peak / n_steps):.2e}")
        out.append(Workload(f"batched_{t}", "gmm_full", d, K,
                            {"weights": w, "means": m, "covs": c}, "rwmh",
                            0.02, n_chains, n_steps, 4 * n_steps, c_tilde, seed,
                            problem_seed))
    return out


def batched_family(n_targets: int = 16, d: int = 8, problem_seed: int = 1006, seed: int = 2006,
                   n_steps: int = 512, n_chains: int = 1 << 16) -> List[Workload]:
    """A family of batched targets of one dimension (the shared learned-mu
    study): d-D full-covariance mixtures as in gmm_full with K uniform in
    {8..16}, n_chains chains each, random-walk MH with sigma 0.02, uniform
    mu, c_tilde by the lifetime rule of batched_uneven.  Target t uses
    Philox target id t."""
    rng = np.random.default_rng(problem_seed)
    out = []
    for t in range(n_targets):
        K = int(rng.integers(8, 17))
        w, m, c = _full_cov_mixture(rng, d, K)
        peak = float((w * (2 * math.pi) ** (-d / 2) / np.sqrt(np.linalg.det(c))).sum())
        c_tilde = float(f"{max(1.0, 8.0 * peak / n_steps):.2e}")
        out.append(Workload(f"family_{t}", "gmm_full", d, K, {"weights": w, "means": m, "covs": c}, "rwmh",
                            0.02, n_chains, n_steps, 4 * n_steps, c_tilde, seed, problem_seed))
    return out


def one_d_three_mode(c: float = 0.25) -> Workload:
    """A 1-D three-mode mixture on [0,1] in the spirit of the paper's
    global-discovery example.  The paper prints no mode locations, so these
    are our own (means 0.2/0.5/0.8, sigma 0.04, equal weights).  ``c`` is the
    inverse expected lifetime; the caller sets c_tilde = c * p_lambda."""
    params = {
        "weights": np.full(3, 1.0 / 3.0),
        "means": np.array([[0.2], [0.5], [0.8]]),
        "sigmas": np.full(3, 0.04),
    }
    return Workload("three_mode_1d", "gmm_iso", 1, 3, params, "rwmh", 0.02,
                    4096, 200, 800, float(c), 2006, 0)


WORKLOADS = {
    "gmm_iso_2d": gmm_iso_2d,
    "gmm_iso_2d_unadjusted": gmm_iso_2d_unadjusted,
    "gmm_full_8d": gmm_full,
    "pss_render_12d": pss_render,
}


def get_workload(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)
