"""Parity of the HIP path's tile-stratified restore runs with the FP64
oracle (the image integrand; each tile its own restore problem with the
target restricted to the tile and mu uniform on it, splats accumulated in
an LDS copy of the workgroup's tile).

Tolerances as for the untiled image workload (test_gpu_parity): chain sums
equal to float32 accuracy for chains whose trajectories meet no near-tie,
image tile sums within 1e-3 (median) of the oracle's, estimates within 3
combined SE of the oracle's and of the truth.
"""
import math

import numpy as np
import pytest

from tests.test_gpu_parity import _say, _single_step_check, _sync

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_07148_amd import restore
    return restore


def _oracle_batch_images(O, wl, prob, B):
    """Batch images of the oracle: tile t's chains split into B ranges."""
    tiles, _ = O.tiles(prob)
    tid = O.tile_of_chain(prob, np.arange(wl.n_chains))
    imgs = np.zeros((B, wl.image[1], wl.image[0]))
    runs = []
    for t in range(len(tiles)):
        lo_t, hi_t = np.flatnonzero(tid == t)[[0, -1]]
        n_t = hi_t + 1 - lo_t
        for b in range(B):
            lo = lo_t + -(-b * n_t // B)
            hi = lo_t + -(-(b + 1) * n_t // B)
            r = O.run(prob, int(lo), int(hi))
            imgs[b] += r.image
            runs.append((int(lo), r))
    return imgs, runs


@pytest.mark.parametrize("n_chains", [8192, 8192 + 77])
def test_tiled_image_and_estimates_match_oracle(R, n_chains):
    """16 tiles x 4 batch images on a 64 x 64 image; 8192 chains (tiles
    aligned with workgroups) and 8269 (workgroups straddle tiles, so part
    of the splats bypass the LDS tile)."""
    from oracle import oracle as O
    from workloads import pss_render
    wl = pss_render(n_chains=n_chains, n_steps=200, image=(64, 64), image_batches=4).with_(tile_px=16)
    _say(f"[tiles {n_chains}] gpu")
    run = R.Run(R.problem_from_workload(wl))
    run.step(wl.n_steps)
    run.drain()
    est = run.estimate()
    mean, se = run.image_estimate()
    img = run.image.cpu().numpy().astype(np.float64)
    arr = {k: v.cpu().numpy() for k, v in run.arrays().items() if k in ("n_done", "t_done")}
    mean = mean.cpu().numpy().astype(np.float64)
    run.close()
    prob = O.Problem(wl)
    oimgs, runs = _oracle_batch_images(O, wl, prob, 4)
    # per-chain sums
    n_o = np.zeros(n_chains, np.int64)
    t_o = np.zeros(n_chains)
    for lo, r in runs:
        n_o[lo:lo + len(r.n_done)] = r.n_done
        t_o[lo:lo + len(r.n_done)] = r.t_done
    same = np.mean((arr["n_done"] == n_o) & (np.abs(arr["t_done"] - t_o) <= 1e-4 * np.maximum(t_o, 1e-30)))
    tiles = lambda im: im.reshape(16, 4, 16, 4).sum(axis=(1, 3))
    rel = [np.abs(tiles(img[b]) - tiles(oimgs[b])) / np.maximum(tiles(oimgs[b]), 1e-30) for b in range(4)]
    med = max(float(np.median(r)) for r in rel)
    _say(f"[tiles {n_chains}] chains with equal sums {same:.4f}; batch-image 4x4-block rel diff median {med:.2e}; "
         f"image total {img.sum():.6g} chain time {arr['t_done'].sum():.6g}")
    assert same > 0.97 and med < 1e-3
    assert abs(img.sum() - arr["t_done"].sum()) <= 1e-4 * arr["t_done"].sum()
    # stratified estimates: the oracle's over the same chains
    full = O.RunResult(n_o, t_o, np.zeros(n_chains), np.zeros(n_chains, np.int32), np.zeros(n_chains),
                       np.zeros(n_chains, np.int64), np.zeros(n_chains, np.int64), np.zeros(n_chains, np.int64),
                       oimgs.sum(axis=0), prob.c_tilde)
    for lo, r in runs:
        full.a_done[lo:lo + len(r.n_done)] = r.a_done
    oest = O.estimate_tiles(prob, full)
    for key in ("p_lambda", "lam_pf", "pi_f"):
        _say(f"[tiles {n_chains}] {key}: gpu {est[key]:.6g} +- {est[key + '_se']:.2g} oracle {oest[key]:.6g} "
             f"+- {oest[key + '_se']:.2g}")
        assert abs(est[key] - oest[key]) < 3 * math.hypot(est[key + "_se"], oest[key + "_se"])
        assert abs(est[key + "_se"] / oest[key + "_se"] - 1) < 0.1
    # the image estimate: c_tilde A_t S_j / N_t per tile, against the oracle's
    oimg = O.image_estimate_tiles(prob, full)
    d = np.abs(tiles(mean) - tiles(oimg)) / np.maximum(tiles(oimg), 1e-30)
    _say(f"[tiles {n_chains}] image estimate 4x4-block rel diff median {np.median(d):.2e}; "
         f"sum {mean.sum():.6g} vs p_lambda {est['p_lambda']:.6g}")
    assert np.median(d) < 1e-3
    assert abs(mean.sum() - est["p_lambda"]) < 1e-3 * est["p_lambda"]


def test_tiled_single_transitions(R):
    from workloads import pss_render
    wl = pss_render(n_chains=16384, image=(128, 128), image_batches=2).with_(tile_px=32)
    k, a, m = _single_step_check(R, wl, warm=5, c_tilde=1.0, label="tiles pss warm", lp_atol=4e-5)
    assert k > 100 and a > 100


def test_tiled_full_size_matches_truth(R):
    """The image workload at full size, 2^20 chains x 256 steps on 512^2
    pixels in 64 x 64 tiles with 16 batch images: estimate against the
    truth, image tiles against the per-pixel truth, and 128 sampled
    chains against the oracle."""
    import json, os
    from workloads import pss_render
    wl = pss_render().with_(tile_px=64)
    truths = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "truths.json")))["pss_render_12d"]
    run = R.Run(R.problem_from_workload(wl))
    run.step(wl.n_steps)
    run.drain()
    est = run.estimate()
    mean, se = run.image_estimate()
    _sync()
    t = truths["tile"]
    tt = np.asarray(truths["tiles"], dtype=np.float64)
    m = mean.cpu().numpy().astype(np.float64)
    tiles = m.reshape(512 // t, t, 512 // t, t).sum(axis=(1, 3))
    rel = (tiles - tt) / tt
    z = (est["p_lambda"] - truths["p_lambda"]) / est["p_lambda_se"]
    _say(f"[tiles full] p_lambda {est['p_lambda']:.6g} +- {est['p_lambda_se']:.2g} truth {truths['p_lambda']:.6g} "
         f"(z {z:.2f}); image {t}x{t}-block rel RMSE {np.sqrt(np.mean(rel ** 2)):.3f}; censored "
         f"{est['tours_censored']}")
    assert abs(z) < 4 and est["tours_censored"] == 0
    # chains spread over the population (and so over the tiles) rerun by the
    # oracle from the same counters, each with its own tile
    arr = {k: v.cpu().numpy() for k, v in run.arrays().items() if k in ("n_done", "t_done")}
    run.close()
    from oracle import oracle as O
    oprob = O.Problem(wl)
    rng = np.random.default_rng(6)
    ids = np.unique(np.concatenate([rng.integers(0, wl.n_chains, 124), [0, 1, wl.n_chains - 2, wl.n_chains - 1]]))
    same = 0
    for c in ids:
        r = O.run(oprob, int(c), int(c) + 1, threads=1)
        same += (int(arr["n_done"][c]) == int(r.n_done[0]) and
                 abs(arr["t_done"][c] - r.t_done[0]) <= 1e-4 * max(1e-30, abs(r.t_done[0])))
    _say(f"[tiles full] sampled chains identical to the oracle: {same}/{len(ids)}")
    assert same >= len(ids) - 2
