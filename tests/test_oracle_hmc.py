"""Pins of the oracle's Hamiltonian Monte Carlo small-step kernel -- no GPU.

HMC is the third local dynamics of the paper's study (Sec. 9: Metropolis,
MALA and HMC, and their restore variants): a momentum rho ~ N(0, I), n
leapfrog steps of size e of the dynamics with potential -log p and unit
mass, accepted with exp(-H(y, rho_n) + H(x, rho_0)), H = -log p + |rho|^2/2.
The pins use facts of the mathematics, not the oracle's code:

* one leapfrog step is the Langevin proposal (MALA) with the same e, and
  the HMC acceptance ratio equals MALA's proposal-density ratio;
* the leapfrog map is reversible (flip the momentum, integrate again, and
  the start comes back) and volume-preserving (unit Jacobian determinant,
  by central differences);
* its energy error is of second order in e;
* HMC leaves pi invariant (exact pi draws stay pi-distributed);
* a whole restore run with HMC local moves matches the erf truth.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import truth
from tests import helpers as H
from workloads import gmm_iso_2d

P_MIN = 1e-4


def _run_transitions(prob, x, n_steps, step0=1):
    n = x.shape[0]
    st = O.States(x.copy(), np.zeros(n), np.zeros(n), np.zeros_like(x))
    chains = np.arange(n)
    out = []
    for s in range(n_steps):
        st, dt, flags, margins = O.transitions(prob, st, step0 + s, chains, recompute=(s == 0))
        out.append((flags, margins))
    return st, out


def test_one_leapfrog_step_is_mala(oracle_lib):
    wl = gmm_iso_2d()
    x = H.sample_pi_iso(wl, 20000, np.random.default_rng(71))
    eps = 0.03
    hmc = O.Problem(wl, c_tilde=0.0, step=eps, local="hmc", n_leapfrog=1)
    mala = O.Problem(wl, c_tilde=0.0, step=eps, local="mala")
    st0 = O.States(x, np.zeros(len(x)), np.zeros(len(x)), np.zeros_like(x))
    a, _, fa, ma = O.transitions(hmc, st0, 3, np.arange(len(x)))
    b, _, fb, mb = O.transitions(mala, st0, 3, np.arange(len(x)))
    near = np.abs(mb[:, 1]) < 1e-9
    assert np.array_equal(fa[~near], fb[~near])
    assert np.count_nonzero(fa & O.FLAG_ACCEPT) > 0.5 * len(x)
    assert np.allclose(a.x, b.x, rtol=0, atol=1e-12)
    # the two acceptance log-ratios agree (ln u_acc minus each)
    fin = np.isfinite(ma[:, 1]) & np.isfinite(mb[:, 1])
    assert np.allclose(ma[fin, 1], mb[fin, 1], rtol=0, atol=1e-9)


def test_leapfrog_is_reversible_and_volume_preserving(oracle_lib):
    wl = gmm_iso_2d()
    prob = O.Problem(wl, local="hmc", n_leapfrog=7, step=0.02)
    rng = np.random.default_rng(72)
    x = H.sample_pi_iso(wl, 20, rng)
    checked = 0
    for q0 in x:
        rho0 = rng.standard_normal(2)
        q1, rho1, _, _, inside = O.leapfrog(prob, q0, rho0, 7, 0.02)
        if not inside:
            continue
        q2, rho2, _, _, inside2 = O.leapfrog(prob, q1, -rho1, 7, 0.02)
        assert inside2
        assert np.allclose(q2, q0, rtol=0, atol=1e-12) and np.allclose(rho2, -rho0, rtol=0, atol=1e-10)
        # Jacobian of (q, rho) -> (q', rho') by central differences
        h = 1e-6
        J = np.zeros((4, 4))
        z0 = np.concatenate([q0, rho0])
        for j in range(4):
            dz = np.zeros(4)
            dz[j] = h
            p_ = O.leapfrog(prob, (z0 + dz)[:2], (z0 + dz)[2:], 7, 0.02)
            m_ = O.leapfrog(prob, (z0 - dz)[:2], (z0 - dz)[2:], 7, 0.02)
            J[:, j] = (np.concatenate([p_[0], p_[1]]) - np.concatenate([m_[0], m_[1]])) / (2 * h)
        assert abs(np.linalg.det(J) - 1.0) < 1e-5
        checked += 1
    assert checked >= 15


def test_leapfrog_energy_error_is_second_order(oracle_lib):
    """Over a fixed trajectory length, halving e divides the energy error
    by about 4 (global error O(e^2))."""
    wl = gmm_iso_2d()
    prob = O.Problem(wl, local="hmc", n_leapfrog=1, step=0.01)
    rng = np.random.default_rng(73)
    x = H.sample_pi_iso(wl, 200, rng)
    rho = rng.standard_normal((200, 2))

    def dH(e, n):
        out = []
        for q0, r0 in zip(x, rho):
            lp0 = O.log_target(prob, q0)[0]
            q1, r1, lp1, _, inside = O.leapfrog(prob, q0, r0, n, e)
            if inside:
                out.append((-lp1 + 0.5 * r1 @ r1) - (-lp0 + 0.5 * r0 @ r0))
        return np.sqrt(np.mean(np.square(out)))

    r = dH(0.004, 5) / dH(0.002, 10)
    assert 3.0 < r < 5.0, r


def test_hmc_is_pi_invariant(oracle_lib):
    """With c_tilde = 0 the HMC chain alone keeps exact pi draws
    pi-distributed (5 leapfrog steps of 0.02, 20 updates)."""
    wl = gmm_iso_2d()
    n = 60000
    x0 = H.sample_pi_iso(wl, n, np.random.default_rng(74))
    prob = O.Problem(wl, c_tilde=0.0, step=0.02, local="hmc", n_leapfrog=5)
    st, out = _run_transitions(prob, x0, 20)
    acc = np.mean([np.mean((f & O.FLAG_ACCEPT) != 0) for f, _ in out])
    assert acc > 0.5
    edges = np.linspace(0, 1, 11)
    obs = H.hist2d(st.x, edges).ravel()
    exp_ = H.iso_cell_masses(wl, edges).ravel()
    exp_ = exp_ / exp_.sum()
    assert H.chi2_pvalue(obs, exp_ * n) > P_MIN


def test_whole_run_with_hmc_moves_matches_erf_truth(oracle_lib):
    wl = gmm_iso_2d().with_(local="hmc", step=0.02, n_leapfrog=5)
    est = O.estimate(O.run(O.Problem(wl), 0, wl.n_chains))
    tr = truth.truths(wl)
    assert est["tours_censored"] == 0
    for key in ("p_lambda", "lam_pf", "pi_f"):
        assert abs(est[key] - tr[key]) < 3 * est[key + "_se"], key
