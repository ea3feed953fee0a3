"""The batched path (many uneven targets, one persistent work-queue launch
captured in a hipGraph) against single-target runs and the oracle."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available()
    from paper_2409_07148_amd import restore
    return restore


def _small_batch(n_targets=12, n_steps=48, lo=200, hi=3000):
    from workloads import batched_uneven
    return batched_uneven(n_targets=n_targets, n_steps=n_steps, chains_lo=lo, chains_hi=hi)


def _sums(batch, t):
    return {k: v.cpu().numpy().copy() for k, v in batch.chain_sums(t).items()}


def test_batch_targets_reproduce_single_target_runs(R):
    """Target i of the batch (Philox target id i) follows exactly the
    trajectories of a single-target run with target id i."""
    wls = _small_batch()
    b = R.Batch(wls, n_steps=wls[0].n_steps)
    b.run()
    for t in (0, 3, 7, 11):
        wl = wls[t]
        run = R.Run(R.problem_from_workload(wl, target_id=t))
        run.step(wl.n_steps)
        run.drain()
        arr = run.arrays()
        got = _sums(b, t)
        assert np.array_equal(got["n_done"], arr["n_done"].cpu().numpy())
        assert np.array_equal(got["t_done"], arr["t_done"].cpu().numpy())
        assert np.array_equal(got["a_done"], arr["a_done"].cpu().numpy())
        est = run.estimate()
        bt = b.estimates()[t]
        # identical per-chain sums; the two reductions use different fixed trees
        assert abs(bt["p_lambda"] / est["p_lambda"] - 1) < 1e-12 and bt["transitions"] == est["transitions"]
        _say(f"[batch vs single] target {t} (d={wl.d}, K={wl.K}, chains {wl.n_chains}): identical")
        run.close()
    b.close()


@pytest.mark.parametrize("buckets", [0, 1])
def test_batch_with_learned_form_mu_reproduces_single_target_runs(R, buckets):
    """Targets of one batch with their own regeneration distribution of the
    learned form (a defensive diagonal mixture built from each target's
    components) next to uniform-mu targets: every target's chains equal a
    single-target run with the same mu and target id, bit for bit, in every
    launch mode and with one or four dimension buckets."""
    from tests import helpers as H
    from workloads import gmm_full
    wls = [gmm_full(d=d, K=K, n_chains=n, n_steps=40, local="rwmh", step=0.02, problem_seed=900 + d + K,
                    c_tilde=ct)
           for d, K, n, ct in ((2, 4, 1500, 30.0), (8, 16, 2100, 1e4), (8, 6, 700, 1e3), (2, 3, 333, 5.0))]
    mus = [H.mixture_mu_from_target(wls[0]), None, H.mixture_mu_from_target(wls[2], beta=0.2), None]
    b = R.Batch(wls, n_steps=40, mus=mus)
    b.set_tiling(buckets=buckets)
    for mode in (R.BATCH_MODE_GRAPH, R.BATCH_MODE_PERSISTENT, R.BATCH_MODE_SEPARATE):
        b.run(mode)
        for t, wl in enumerate(wls):
            run = R.Run(R.problem_from_workload(wl, target_id=t, mu=mus[t]))
            run.step(wl.n_steps)
            run.drain()
            arr = run.arrays()
            got = _sums(b, t)
            for k in ("n_done", "t_done", "a_done"):
                assert np.array_equal(got[k], arr[k].cpu().numpy()), (mode, t, k)
            if mode == R.BATCH_MODE_GRAPH:
                est = run.estimate()
                bt = b.estimates()[t]
                assert abs(bt["p_lambda"] / est["p_lambda"] - 1) < 1e-12 and bt["kills"] == est["kills"]
                _say(f"[batch learned mu buckets={buckets}] target {t} (d={wl.d}, mu "
                     f"{'learned form' if mus[t] is not None else 'uniform'}): identical; p_lambda "
                     f"{est['p_lambda']:.4g}, kill rate {est['kill_rate']:.3f}")
            run.close()
    b.close()


def test_batch_largest_learned_form_mu(R):
    """The largest learned-form mu a batched workgroup copies to LDS: 64
    components at d = 16 (and at d = 8), each target's own mixture with a
    defensive share.  The 8-D target equals its single-target run bit for
    bit; the 16-D target, which has no single-target kernel with a learned
    mu, is compared with the oracle chain by chain on sampled chains.  Both
    the persistent (graph) and the one-launch-per-target kernels."""
    from tests import helpers as H
    from tests import chain_parity as CP
    from workloads import gmm_full
    from oracle import oracle as O
    # c~ = 1: about half the transitions kill, the rest are local moves
    wls = [gmm_full(d=16, K=64, n_chains=900, n_steps=40, local="rwmh", step=0.01, problem_seed=1080,
                    c_tilde=1.0),
           gmm_full(d=8, K=64, n_chains=1300, n_steps=40, local="rwmh", step=0.02, problem_seed=1072,
                    c_tilde=1.0)]
    mus = [H.mixture_mu_from_target(w) for w in wls]
    b = R.Batch(wls, n_steps=40, mus=mus)
    ids = np.unique(np.concatenate([np.random.default_rng(8).integers(0, wls[0].n_chains, 30), [0, 899]]))
    oprob = O.Problem(wls[0], mu=mus[0], target_id=0)
    rs = [O.run(oprob, int(c), int(c) + 1, threads=1) for c in ids]
    cat = lambda f: np.concatenate([getattr(r, f) for r in rs])
    ores = O.RunResult(cat("n_done"), cat("t_done"), cat("a_done"), cat("censored"), cat("t_censored"),
                       cat("transitions"), cat("accepts"), cat("kills"), None, oprob.c_tilde,
                       min_margin=np.concatenate([r.min_margin for r in rs]))
    run = R.Run(R.problem_from_workload(wls[1], target_id=1, mu=mus[1]))
    run.step(wls[1].n_steps)
    run.drain()
    arr = {k: v.cpu().numpy() for k, v in run.arrays().items()}
    run.close()
    for mode in (R.BATCH_MODE_GRAPH, R.BATCH_MODE_SEPARATE):
        b.run(mode)
        got = _sums(b, 0)
        CP.check_chain_sums({k: got[k][ids] for k in ("n_done", "t_done", "a_done")}, ores, wls[0], mu=mus[0],
                            say=_say, label=f"batch d=16 64-component mu, mode {mode}")
        got = _sums(b, 1)
        for k in ("n_done", "t_done", "a_done"):
            assert np.array_equal(got[k], arr[k]), (mode, k)
        est = b.estimates()
        _say(f"[batch largest mu] mode {mode}: d=16 kill rate {est[0]['kill_rate']:.3f}, "
             f"tours {est[0]['tours_done']}; d=8 identical to its single-target run")
    b.close()


def test_batch_results_do_not_depend_on_tiling_or_mode(R):
    wls = _small_batch(n_targets=10)
    b = R.Batch(wls, n_steps=wls[0].n_steps)
    b.run()
    ref = [_sums(b, t) for t in range(len(wls))]
    ref_est = b.estimates()
    for block, order, buckets, mode in [(64, 0, 0, R.BATCH_MODE_GRAPH), (128, 1, 1, R.BATCH_MODE_GRAPH),
                                        (256, 0, 1, R.BATCH_MODE_PERSISTENT), (64, 1, 0, R.BATCH_MODE_SEPARATE),
                                        (256, 1, 1, R.BATCH_MODE_SEPARATE)]:
        b.set_tiling(block, order, buckets)
        b.run(mode)
        est = b.estimates()
        for t in range(len(wls)):
            got = _sums(b, t)
            for k in ref[t]:
                assert np.array_equal(ref[t][k], got[k]), (block, order, buckets, mode, t, k)
            assert est[t]["p_lambda"] == ref_est[t]["p_lambda"]
            assert est[t]["transitions"] == ref_est[t]["transitions"]
    b.close()


def test_graph_replays_with_eager_work_between(R):
    """Replays of the captured pass, with unrelated eager GPU work and
    synchronisations between them, each give the eager pass's results."""
    import torch
    wls = _small_batch(n_targets=6)
    b = R.Batch(wls, n_steps=wls[0].n_steps)
    b.run(R.BATCH_MODE_PERSISTENT)
    ref = b.estimates()
    for rep in range(3):
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()
        b.run(R.BATCH_MODE_GRAPH)
        est = b.estimates()
        for t in range(len(wls)):
            assert est[t]["p_lambda"] == ref[t]["p_lambda"], (rep, t)
            assert est[t]["transitions"] == ref[t]["transitions"]
    b.close()


def test_autotune_picks_and_caches_a_tiling(R, tmp_path):
    wls = _small_batch(n_targets=8)
    b = R.Batch(wls, n_steps=wls[0].n_steps)
    cache = str(tmp_path / "tiling.json")
    t1, ms1 = b.autotune(cache)
    assert os.path.exists(cache) and ms1 > 0
    b2 = R.Batch(wls, n_steps=wls[0].n_steps)
    t2, ms2 = b2.autotune(cache)
    assert (t1.block_size, t1.order, t1.buckets) == (t2.block_size, t2.order, t2.buckets)
    assert abs(ms2 - ms1) < 1e-3  # the cache stores the time to 1e-4 ms
    _say(f"[autotune] chose {t1.as_dict()} at {ms1:.3f} ms")
    b.close()
    b2.close()


def test_full_batch_sampled_chains_match_oracle(R):
    """The full 256-target batch (log-uniform 1K..256K chains, d 2..16, K
    2..32, 256 steps): chains of a few targets rerun by the oracle from the
    same counters."""
    from workloads import batched_uneven
    from oracle import oracle as O
    wls = batched_uneven()
    _say(f"[full batch] {len(wls)} targets, {sum(w.n_chains for w in wls)} chains")
    b = R.Batch(wls, n_steps=256)
    b.run()
    est = b.estimates()
    _say(f"[full batch] transitions {sum(e['transitions'] for e in est)}, "
         f"censored {sum(e['tours_censored'] for e in est)}")
    rng = np.random.default_rng(5)
    picks = [int(i) for i in rng.choice(len(wls), 4, replace=False)]
    picks.append(int(np.argmax([w.d * 100 + w.K for w in wls])))
    # holding times below the float32 range (~1e-38; c_tilde reaches 1e17
    # here) are zero on the GPU and tiny in the FP64 oracle: per chain at
    # most ~1000 of them, hence the absolute floor
    floor = 1e-35
    same = total = 0
    shown = 0
    for t in picks:
        wl = wls[t]
        got = _sums(b, t)
        oprob = O.Problem(wl, target_id=t)
        for c in rng.integers(0, wl.n_chains, 12):
            r = O.run(oprob, int(c), int(c) + 1, threads=1)
            total += 1
            ok = (int(got["n_done"][c]) == int(r.n_done[0]) and
                  abs(got["t_done"][c] - r.t_done[0]) <= 1e-4 * abs(r.t_done[0]) + floor)
            same += ok
            if not ok and shown < 6:
                shown += 1
                _say(f"[full batch] mismatch target {t} chain {c}: n {got['n_done'][c]} vs {r.n_done[0]}, "
                     f"T {got['t_done'][c]:.6e} vs {r.t_done[0]:.6e}")
        _say(f"[full batch] target {t}: d={wl.d} K={wl.K} chains={wl.n_chains} c~={wl.c_tilde:g} "
             f"p_lambda {est[t]['p_lambda']:.4g} +- {est[t]['p_lambda_se']:.2g}")
    _say(f"[full batch] sampled chains identical to the oracle: {same}/{total}")
    assert same >= total - 2
    b.close()
