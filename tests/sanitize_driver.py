"""Driver of the sanitizer runs (tests/test_sanitizers.py), run in a child
process with the sanitizer runtime preloaded.

    python tests/sanitize_driver.py oracle <liboracle built with ASan/UBSan>
    python tests/sanitize_driver.py host <librestore with host-side ASan/UBSan>

`oracle` drives the FP64 oracle through its whole-run, single-transition,
density, tile, MH, HMC and unadjusted-jump entry points on small inputs.
`host` drives the library's host-side validation -- the descriptor checks
and layout arithmetic of restore_state_bytes, restore_batch_state_bytes,
restore_mlp_param_count and the NLL and Adam argument checks -- with valid
and invalid descriptors; it launches no device work."""
import ctypes as C
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def drive_oracle(path):
    from oracle import oracle as O
    from tests import helpers as H
    from workloads import gmm_full, gmm_iso_2d, gmm_iso_2d_unadjusted, pss_render
    with O.use_library(path):
        wl = gmm_iso_2d(n_chains=256, n_steps=40)
        O.estimate(O.run(O.Problem(wl), 0, 256, threads=2))
        O.run(O.Problem(wl, c_tilde=0.0, large_step_prob=0.3, burn_in=10), 0, 64, n_steps=50)
        O.run(O.Problem(wl.with_(local="hmc", n_leapfrog=3), step=0.02), 0, 64)
        O.run(O.Problem(gmm_iso_2d_unadjusted(n_chains=64, n_steps=30)), 0, 64)
        w8 = gmm_full(n_chains=128, n_steps=20)
        st = O.init_states(O.Problem(w8), np.arange(128))
        O.transitions(O.Problem(w8), st, 3, np.arange(128))
        mu = H.mixture_mu_from_target(w8)
        O.run(O.Problem(w8, mu=mu, c_tilde=1.0), 0, 64)
        O.log_mu(O.Problem(w8, mu=mu), np.random.default_rng(0).random((50, 8)))
        wp = pss_render(n_chains=64, n_steps=20, image=(32, 32), image_batches=2)
        O.run(O.Problem(wp), 0, 64)
        O.run(O.Problem(wp.with_(tile_px=8)), 0, 64)
        O.log_inflow(O.Problem(gmm_iso_2d_unadjusted()), np.random.default_rng(1).random((20, 2)))


def drive_host(path):
    from paper_2409_07148_amd import restore as R
    from workloads import batched_uneven, gmm_full, gmm_iso_2d, gmm_iso_2d_unadjusted, pss_render
    lib = R._load(path)
    ok, refused = 0, 0

    def state_bytes(p):
        n = C.c_size_t(0)
        return lib.restore_state_bytes(C.byref(p.target), C.byref(p.mu), C.byref(p.local), C.byref(p.cfg),
                                       C.byref(n)), n.value

    valid = [R.problem_from_workload(gmm_iso_2d()), R.problem_from_workload(gmm_full()),
             R.problem_from_workload(gmm_full(n_chains=3000)),
             R.problem_from_workload(gmm_full(d=16, K=64, n_chains=777)),
             R.problem_from_workload(gmm_iso_2d_unadjusted()),
             R.problem_from_workload(gmm_iso_2d(), local="hmc", n_leapfrog=5),
             R.problem_from_workload(gmm_iso_2d(), c_tilde=0.0, large_step_prob=0.3),
             R.problem_from_workload(pss_render()),
             R.problem_from_workload(pss_render(n_chains=8192, image=(64, 64), image_batches=4), tile_px=16),
             R.problem_from_workload(gmm_iso_2d(), first_chain=123456, flags=R.FLAG_INLINE_RNG)]
    for p in valid:
        st, n = state_bytes(p)
        assert st == 0 and n > 0, (st, lib.restore_last_error())
        ok += 1
    mutations = [("c_tilde", -1.0), ("n_chains", 0), ("n_chains", 1 << 40), ("drain_cap", -3), ("block_size", 96),
                 ("first_chain", -1), ("image_batches", 5), ("tile_px", 3), ("c_tilde", float("nan"))]
    for field, value in mutations:
        p = R.problem_from_workload(gmm_full(n_chains=1000))
        setattr(p.cfg, field, value)
        st, _ = state_bytes(p)
        assert st < 0 and lib.restore_last_error(), (field, value)
        refused += 1
    for field, value in [("dim", 0), ("dim", 17), ("n_comp", 0), ("n_comp", 65), ("kind", 9), ("params_count", 3)]:
        p = R.problem_from_workload(gmm_full(n_chains=1000))
        setattr(p.target, field, value)
        st, _ = state_bytes(p)
        assert st < 0, (field, value)
        refused += 1
    p = R.problem_from_workload(gmm_full(n_chains=1000))
    p._params[5] = float("nan")
    assert state_bytes(p)[0] == R.E_NONFINITE
    for kind, step, lsp, nl in [(9, 0.01, 0.0, 0), (0, -1.0, 0.0, 0), (0, 0.01, 1.5, 0), (2, 0.01, 0.0, 0),
                                (2, 0.01, 0.0, 65), (1, 0.0, 0.0, 0)]:
        p = R.problem_from_workload(gmm_full(n_chains=1000))
        p.local = R.restore_local_kernel(kind, step, lsp, nl)
        assert state_bytes(p)[0] < 0, (kind, step, lsp, nl)
        refused += 1
    n = C.c_size_t(0)
    assert lib.restore_state_bytes(None, None, None, None, C.byref(n)) < 0
    # batches
    wls = batched_uneven()[:12]
    probs = [R.problem_from_workload(w, target_id=i) for i, w in enumerate(wls)]
    T = (R.restore_target * len(probs))(*[p.target for p in probs])
    L = (R.restore_local_kernel * len(probs))(*[p.local for p in probs])
    G = (R.restore_config * len(probs))(*[p.cfg for p in probs])
    assert lib.restore_batch_state_bytes(len(probs), T, L, G, None, C.byref(n)) == 0 and n.value > 0
    G[3].c_tilde = 0.0
    assert lib.restore_batch_state_bytes(len(probs), T, L, G, None, C.byref(n)) < 0
    G[3].c_tilde = 1.0
    G[4].first_chain = -2
    assert lib.restore_batch_state_bytes(len(probs), T, L, G, None, C.byref(n)) < 0
    assert lib.restore_batch_state_bytes(0, T, L, G, None, C.byref(n)) < 0
    # the learned part's argument checks (no device work)
    shape = R.restore_mlp_shape(12, 64, 64, 8)
    npar, nact = C.c_int64(0), C.c_int64(0)
    assert lib.restore_mlp_param_count(C.byref(shape), C.byref(npar), C.byref(nact)) == 0
    assert lib.restore_mlp_param_count(C.byref(R.restore_mlp_shape(12, 64, 65, 8)), C.byref(npar), None) < 0
    assert lib.restore_gmm_nll_workspace_bytes(C.byref(n)) == 0 and n.value > 0
    assert lib.restore_gmm_nll(0, 8, 0.1, None, None, None, 10, None, None, None, 0, None) < 0
    assert lib.restore_adam_step(None, None, None, None, 10, 1, 1e-3, 0.9, 0.999, 1e-8, None) < 0
    print(f"host validation: {ok} valid descriptors accepted, {refused} invalid ones refused", flush=True)


if __name__ == "__main__":
    {"oracle": drive_oracle, "host": drive_host}[sys.argv[1]](sys.argv[2])
    print("driver done", flush=True)
