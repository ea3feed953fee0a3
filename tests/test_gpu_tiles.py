"""Parity of the HIP path's tile-stratified restore runs with the FP64
oracle (the image integrand; each tile its own restore problem with the
target restricted to the tile and mu uniform on it, splats accumulated in
an LDS copy of the workgroup's tile).

Tolerances as for the untiled image workload (test_gpu_parity and
tests/chain_parity.py): every chain whose trajectory meets no near-tie has
the oracle's tour count and its sums within the float32 bounds; batch images
and the image estimate agree pixel by pixel within theirs (a near-tie chain
splats only into its own tile, so the tiles of near-tie chains are left out
and counted); estimates within 3 combined SE of the oracle's and of the
truth.
"""
import math

import numpy as np
import pytest

from tests import chain_parity as CP
from tests.test_gpu_parity import _oracle_chains, _say, _single_step_check, _sync

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_07148_amd import restore
    return restore


def _oracle_batch_images(O, wl, prob, B):
    """Batch images of the oracle (tile t's chains split into B ranges),
    with their splat counts and edge masses, the per-chain results of the
    whole population, and the batch of every chain."""
    tiles, _ = O.tiles(prob)
    tid = O.tile_of_chain(prob, np.arange(wl.n_chains))
    shape = (B, wl.image[1], wl.image[0])
    imgs, cnts, edges = np.zeros(shape), np.zeros(shape), np.zeros(shape)
    n = wl.n_chains
    full = O.RunResult(np.zeros(n, np.int64), np.zeros(n), np.zeros(n), np.zeros(n, np.int32), np.zeros(n),
                       np.zeros(n, np.int64), np.zeros(n, np.int64), np.zeros(n, np.int64), None, prob.c_tilde,
                       min_margin=np.zeros((n, 4)))
    batch = np.zeros(n, np.int64)
    for t in range(len(tiles)):
        lo_t, hi_t = np.flatnonzero(tid == t)[[0, -1]]
        n_t = hi_t + 1 - lo_t
        for b in range(B):
            lo = lo_t + -(-b * n_t // B)
            hi = lo_t + -(-(b + 1) * n_t // B)
            r = O.run(prob, int(lo), int(hi))
            imgs[b] += r.image
            cnts[b] += r.image_count
            edges[b] += r.image_near
            for f in ("n_done", "t_done", "a_done", "censored", "t_censored", "transitions", "min_margin"):
                getattr(full, f)[lo:hi] = getattr(r, f)
            batch[lo:hi] = b
    full.image = imgs.sum(axis=0)
    return imgs, cnts, edges, full, tid, batch


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
    arr = {k: v.cpu().numpy() for k, v in run.arrays().items() if k in ("n_done", "t_done", "a_done")}
    mean = mean.cpu().numpy().astype(np.float64)
    run.close()
    prob = O.Problem(wl)
    oimgs, cnts, edges, full, tid, batch = _oracle_batch_images(O, wl, prob, 4)
    m = CP.check_chain_sums({k: arr[k] for k in ("n_done", "t_done", "a_done")}, full, wl, say=_say,
                            label=f"tiles {n_chains}")
    assert abs(img.sum() - arr["t_done"].sum()) <= 1e-4 * arr["t_done"].sum()
    # pixels of the tiles whose chains (in that batch image) saw no near-tie
    tiles, _ = O.tiles(prob)
    px_tile = np.zeros(wl.image[::-1], np.int64)
    for t, (x0, x1, y0, y1) in enumerate(tiles):
        px_tile[y0:y1, x0:x1] = t
    eps = CP.eps_dt(wl)
    for b in range(4):
        bad_tiles = np.unique(tid[m["near"] & (batch == b)])
        keep = ~np.isin(px_tile, bad_tiles)
        CP.check_image(img[b][keep], oimgs[b][keep], cnts[b][keep], edges[b][keep], eps, say=_say,
                       label=f"tiles {n_chains} batch {b} ({len(bad_tiles)} tiles with near-tie chains left out)")
    # stratified estimates: the oracle's over the same chains
    oest = O.estimate_tiles(prob, full)
    for key in ("p_lambda", "lam_pf", "pi_f"):
        _say(f"[tiles {n_chains}] {key}: gpu {est[key]:.6g} +- {est[key + '_se']:.2g} oracle {oest[key]:.6g} "
             f"+- {oest[key + '_se']:.2g}")
        assert abs(est[key] - oest[key]) < 3 * math.hypot(est[key + "_se"], oest[key + "_se"])
        assert abs(est[key + "_se"] / oest[key + "_se"] - 1) < 0.1
    # the image estimate c_tilde A_t S_j / N_t per tile, against the
    # oracle's, pixel by pixel in the tiles without near-tie chains (N_t is
    # then exact and S_j a float32 sum over the batches)
    oimg = O.image_estimate_tiles(prob, full)
    bad_tiles = np.unique(tid[m["near"]])
    keep = ~np.isin(px_tile, bad_tiles)
    CP.check_image(mean[keep], oimg[keep], cnts.sum(axis=0)[keep] + 4, oimg[keep] / np.maximum(
        oimgs.sum(axis=0)[keep], 1e-300) * edges.sum(axis=0)[keep], eps + 2.0 ** -23, say=_say,
        label=f"tiles {n_chains} image estimate ({len(bad_tiles)} tiles left out)")
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
    arr = {k: v.cpu().numpy() for k, v in run.arrays().items() if k in ("n_done", "t_done", "a_done")}
    run.close()
    from oracle import oracle as O
    rng = np.random.default_rng(6)
    ids = np.unique(np.concatenate([rng.integers(0, wl.n_chains, 124), [0, 1, wl.n_chains - 2, wl.n_chains - 1]]))
    ores = _oracle_chains(O.Problem(wl), ids)
    CP.check_chain_sums({k: arr[k][ids] for k in ("n_done", "t_done", "a_done")}, ores, wl, say=_say,
                        label="tiles full sampled chains")
