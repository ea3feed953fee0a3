"""One chain population run as several chain ranges (restore_config
.first_chain), on one GPU: the part of sharding over devices that one GPU
can show.  Tours spawned from mu are independent (Sec. 1), and every
random number of chain c is drawn with Philox counter word first_chain + c,
so runs over the ranges [c0, c1) of a population give exactly the chains
of one run over all of them: the per-chain sums are compared bit for bit,
and a range is compared with the oracle's run of the same global chains.
"""
import numpy as np
import pytest

from tests import chain_parity as CP
from tests.test_gpu_parity import _say

pytestmark = pytest.mark.gpu

KEYS = ("n_done", "t_done", "a_done", "status", "t_cur")


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_07148_amd import restore
    return restore


def _run(R, wl, lo, hi, **kw):
    run = R.Run(R.problem_from_workload(wl, n_chains=hi - lo, first_chain=lo, **kw))
    run.step(wl.n_steps)
    run.drain()
    est = run.estimate()
    arr = {k: v.cpu().numpy().copy() for k, v in run.arrays().items() if k in KEYS}
    run.close()
    return est, arr


@pytest.mark.parametrize("which", ["gmm_iso_2d", "gmm_full_8d"])
def test_chain_ranges_reproduce_the_whole_population(R, which):
    from oracle import oracle as O
    from workloads import gmm_full, gmm_iso_2d
    wl = {"gmm_iso_2d": lambda: gmm_iso_2d(),
          "gmm_full_8d": lambda: gmm_full(n_chains=20000, n_steps=128)}[which]()
    C = wl.n_chains
    est, ref = _run(R, wl, 0, C)
    for k in (2, 4):
        # uneven ranges, none aligned with a workgroup
        cuts = sorted({0, C} | {int(C * (i / k) + 37 * i) for i in range(1, k)})
        parts = [_run(R, wl, lo, hi) for lo, hi in zip(cuts[:-1], cuts[1:])]
        for key in KEYS:
            got = np.concatenate([a[key] for _, a in parts])
            assert np.array_equal(got, ref[key]), (k, key)
        assert sum(e["transitions"] for e, _ in parts) == est["transitions"]
        assert sum(e["tours_done"] for e, _ in parts) == est["tours_done"]
        _say(f"[shard {which}] {k} ranges {cuts}: every chain bit-identical to the whole run")
    # a range in the middle against the oracle's run of the same global chains
    lo, hi = C // 3, C // 3 + 1500
    _, arr = _run(R, wl, lo, hi)
    ores = O.run(O.Problem(wl), lo, hi)
    CP.check_chain_sums(arr, ores, wl, say=_say, label=f"shard {which} chains {lo}..{hi} vs oracle")


def test_batch_targets_with_chain_offsets(R):
    """Batched targets with a first_chain each follow the single-target runs
    with the same offset and target id bit for bit."""
    from workloads import batched_uneven
    wls = [w.with_(n_chains=min(w.n_chains, 3000)) for w in batched_uneven()[:3]]
    firsts = [0, 5000, 123457]
    b = R.Batch(wls, n_steps=wls[0].n_steps, first_chains=firsts)
    b.run(R.BATCH_MODE_PERSISTENT)
    b.estimates()
    for i, (w, f) in enumerate(zip(wls, firsts)):
        got = {k: v.cpu().numpy() for k, v in b.chain_sums(i).items()}
        run = R.Run(R.problem_from_workload(w, target_id=i, first_chain=f))
        run.step(w.n_steps)
        run.drain()
        ref = {k: v.cpu().numpy() for k, v in run.arrays().items() if k in ("n_done", "t_done", "a_done")}
        run.close()
        for k in ("n_done", "t_done", "a_done"):
            assert np.array_equal(got[k], ref[k]), (i, k)
    b.close()
