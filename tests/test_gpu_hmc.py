"""Parity of the HIP path's Hamiltonian Monte Carlo small-step kernel with
the FP64 oracle (the third local dynamics of the paper's study, Sec. 9).

Tolerances as for the other kernels (test_gpu_parity), except moved
states: the leapfrog adds n position steps of size e |rho| in float32, so
the end point carries up to n roundings of a value below 1 (2^-24 each)
plus the propagated float32 error of the n gradients (|e^2 dg| per step,
dg ~1e-6 |g|): with the tested n <= 8 (e = 0.005, 8-D) and n = 5 (e = 0.02,
2-D, |g| <= ~100) that is below 5e-7 + 2e-7, under the 1e-6 bar.
"""
import math

import numpy as np
import pytest

from tests import chain_parity as CP
from tests.test_gpu_parity import _gpu_run, _oracle_chains, _pi_draws, _say, _single_step_check
from tests.test_gpu_mh import _mh_step_check

pytestmark = pytest.mark.gpu

X_TOL = 1e-6


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_07148_amd import restore
    return restore


def _hmc(wl, step, n):
    return wl.with_(local="hmc", step=step, n_leapfrog=n)


def test_hmc_single_transitions_2d(R):
    from workloads import gmm_iso_2d
    wl = _hmc(gmm_iso_2d(n_chains=20000), 0.02, 5)
    k, a, m = _single_step_check(R, wl, x_init=_pi_draws(wl, wl.n_chains, 81), label="hmc 2d pi", x_tol=X_TOL)
    assert a > 5000
    k, a, m = _single_step_check(R, wl, warm=6, label="hmc 2d warm", x_tol=X_TOL)
    assert k > 1000 and a > 1000


@pytest.mark.parametrize("c_tilde", [1e5, 3.34e7])
def test_hmc_single_transitions_8d(R, c_tilde):
    from workloads import gmm_full
    wl = _hmc(gmm_full(n_chains=8192), 0.005, 8)
    k, a, m = _single_step_check(R, wl, x_init=_pi_draws(wl, wl.n_chains, 82), c_tilde=c_tilde,
                                 label=f"hmc 8d pi c={c_tilde:g}", x_tol=X_TOL)
    assert a > 1000
    _single_step_check(R, wl, warm=4, c_tilde=c_tilde, label=f"hmc 8d warm c={c_tilde:g}", x_tol=X_TOL)


@pytest.mark.parametrize("d,K,n", [(16, 64, 3), (1, 3, 8), (13, 7, 1)])
def test_hmc_single_transitions_extreme_shapes(R, d, K, n):
    from workloads import gmm_full
    wl = _hmc(gmm_full(d=d, K=K, n_chains=4096, problem_seed=4000 + d * 100 + K), 0.004, n)
    x0 = _pi_draws(wl, wl.n_chains, 83)
    for lds in (False, True):
        _single_step_check(R, wl, x_init=x0, c_tilde=1e3, label=f"hmc d{d} K{K} n{n} pi lds={lds}", lds=lds,
                           x_tol=X_TOL)


def test_hmc_mh_chain_with_large_steps(R):
    """The MH chain M^l with HMC small steps and large steps from mu."""
    from workloads import gmm_iso_2d
    wl = _hmc(gmm_iso_2d(n_chains=8192), 0.02, 5)
    n_large, n_large_acc = _mh_step_check(R, wl, 0.3, _pi_draws(wl, wl.n_chains, 84), label="hmc mh 2d",
                                          x_tol=X_TOL)
    assert n_large > 1000 and n_large_acc > 0


def test_hmc_whole_run_2d_matches_oracle_and_truth(R):
    from oracle import oracle as O, truth
    from workloads import gmm_iso_2d
    wl = _hmc(gmm_iso_2d(), 0.02, 5)
    _say("[hmc run 2d] gpu")
    est, arr = _gpu_run(R, wl)
    ores = O.run(O.Problem(wl), 0, wl.n_chains)
    oest = O.estimate(ores)
    tr = truth.truths(wl)
    for key in ("p_lambda", "lam_pf", "pi_f"):
        _say(f"[hmc run 2d] {key}: gpu {est[key]:.6g} +- {est[key + '_se']:.2g}  oracle {oest[key]:.6g}  "
             f"truth {tr[key]:.6g}")
        assert abs(est[key] - oest[key]) < 3 * math.hypot(est[key + "_se"], oest[key + "_se"])
        assert abs(est[key] - tr[key]) < 3 * est[key + "_se"]
    CP.check_chain_sums(arr, ores, wl, say=_say, label="hmc run 2d")
    _say(f"[hmc run 2d] accept rate {est['accept_rate']:.3f}")
    assert est["tours_censored"] == 0


def test_hmc_full_size_8d_sampled_chains_match_oracle(R):
    """The 8-D workload with HMC moves (e = 0.005, 8 leapfrog steps) at its
    full size; 96 chains spread over the population rerun by the oracle."""
    from oracle import oracle as O
    from workloads import gmm_full
    wl = _hmc(gmm_full(), 0.005, 8)
    _say("[hmc full 8d] gpu run 2^20 x 512")
    est, arr = _gpu_run(R, wl)
    rng = np.random.default_rng(85)
    ids = np.unique(np.concatenate([rng.integers(0, wl.n_chains, 92), [0, 1, wl.n_chains - 2, wl.n_chains - 1]]))
    ores = _oracle_chains(O.Problem(wl), ids)
    _say(f"[hmc full 8d] transitions {est['transitions']} accept rate {est['accept_rate']:.3f} kill rate "
         f"{est['kill_rate']:.6f}")
    CP.check_chain_sums({k: arr[k][ids] for k in ("n_done", "t_done", "a_done")}, ores, wl, say=_say,
                        label="hmc full 8d sampled chains")
