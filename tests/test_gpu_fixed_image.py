"""Fixed-point image sums (RESTORE_FLAG_IMAGE_FIXED) through the C ABI.

Every splat adds its float32 dt rounded to a multiple of 2^-32 to a 64-bit
integer per pixel.  Integer addition is exact and commutes, so:
  * the image is the same bit for bit whatever the workgroup size, the LDS
    staging, the split of the steps into restore_step calls or the order in
    which the atomics land (compared with ==);
  * against the oracle's float64 image of the same chains the only error
    left is that of each dt (eps of tests/chain_parity.py), the rounding of
    each splat to 2^-32 (half a unit per step in the pixel), the final
    float32 rounding of the published image (2^-24 of the pixel) and the
    splats whose state lies at a pixel edge (the oracle's image_near): no
    term for the order of float32 additions, which bounds the float image.
"""
import sys

import numpy as np
import pytest

from tests import chain_parity as CP

pytestmark = pytest.mark.gpu


def _sync():
    import torch
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2409_07148_amd import restore
    return restore


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _run(R, wl, splits, drain=True, **kw):
    run = R.Run(R.problem_from_workload(wl, **kw))
    for n in splits:
        run.step(n)
    if drain:
        run.drain()
    _sync()
    img = run.image.clone()
    arr = {k: v.clone() for k, v in run.arrays().items()}
    run.close()
    return img, arr


def test_fixed_image_is_the_same_bit_for_bit(R):
    """2^16 chains x 150 steps of the 12-D image integrand, 4 batch images
    of 256 x 256: the fixed-point image of the default launch equals, bit for
    bit, those of 64- and 128-thread workgroups, LDS-staged parameters, the
    steps split 37 + 113 and a second identical run; the chains equal those
    of the float-image run; the float image of the default binned splats
    agrees within its order-of-additions bound; the image total equals the
    tour time within the float32 rounding of the tour sums."""
    import torch
    from workloads import pss_render
    wl = pss_render(n_chains=1 << 16, n_steps=150, image=(256, 256), image_batches=4)
    F = R.FLAG_IMAGE_FIXED
    ref_img, ref_arr = _run(R, wl, [150], flags=F)
    variants = {"again": ([150], {"flags": F}),
                "block64": ([150], {"flags": F, "block_size": 64}),
                "block128_lds": ([150], {"flags": F, "block_size": 128, "lds": True}),
                "split": ([37, 113], {"flags": F})}
    for name, (splits, kw) in variants.items():
        img, arr = _run(R, wl, splits, **kw)
        same = torch.equal(img, ref_img)
        _say(f"[fixed image] {name}: bit-identical {same}")
        assert same, name
        for k in ("x", "logp", "t_done", "a_done", "n_done", "status"):
            assert torch.equal(arr[k], ref_arr[k]), (name, k)
    flt_img, flt_arr = _run(R, wl, [150])
    for k in ("x", "logp", "t_done", "a_done", "n_done", "status"):
        assert torch.equal(flt_arr[k], ref_arr[k]), k
    a, b = ref_img.double().cpu().numpy(), flt_img.double().cpu().numpy()
    n_terms = (1 << 16) * 160 / (256 * 256 * 4)
    bound = 2 * (8 * n_terms + 1) * 2.0 ** -24 * np.maximum(a, b) + 1e-30
    _say(f"[fixed image] vs float image: max err/bound {float((np.abs(a - b) / bound).max()):.3f}")
    assert np.all(np.abs(a - b) <= bound)
    cens = (ref_arr["status"].cpu().numpy() & R.ST_CENSORED) != 0
    t_all = float(ref_arr["t_done"].double().sum()) + float(ref_arr["t_cur"].cpu().numpy()[cens].astype(np.float64).sum())
    steps = float(wl.n_chains) * (wl.n_steps + wl.drain_cap)
    _say(f"[fixed image] image total {a.sum():.9g} tour time {t_all:.9g}")
    assert abs(a.sum() - t_all) <= 1e-5 * t_all + steps * 2.0 ** -32


def test_fixed_image_matches_oracle_pixel_by_pixel(R):
    """8192 chains x 200 steps, 4 batch images of 128 x 128: each batch
    image, over the chains without a near-tie (clean sub-ranges run on
    their own with their global chain ids), equals the oracle's float64
    image within eps per pixel value, half a 2^-32 unit per splat, the
    final float32 rounding and the edge mass -- no order-of-additions
    term."""
    from workloads import pss_render
    from oracle import oracle as O
    wl = pss_render(n_chains=8192, n_steps=200, image=(128, 128), image_batches=4)
    F = R.FLAG_IMAGE_FIXED
    img, arr = _run(R, wl, [wl.n_steps], flags=F)
    img = img.double().cpu().numpy()
    arr = {k: v.cpu().numpy() for k, v in arr.items()}
    eps = CP.eps_dt(wl)
    worst = 0.0
    for b, (lo, hi) in enumerate(O.batch_ranges(wl.n_chains, 4)):
        ores = O.run(O.Problem(wl), lo, hi)
        m = CP.check_chain_sums({k: arr[k][lo:hi] for k in ("n_done", "t_done", "a_done")}, ores, wl,
                                say=_say, label=f"fixed image batch {b}")
        g, o, cnt, edge = img[b], ores.image, ores.image_count.astype(np.float64), ores.image_near
        if m["near"].any():
            g = o = cnt = edge = None
            for c0, c1 in CP.clean_ranges(m["near"], lo):
                gi, _ = _run(R, wl, [wl.n_steps], flags=F, n_chains=c1 - c0, image_batches=0, first_chain=c0)
                r = O.run(O.Problem(wl), c0, c1)
                if g is None:
                    g, o, cnt, edge = gi.double().cpu().numpy(), r.image.copy(), \
                        r.image_count.astype(np.float64), r.image_near.copy()
                else:
                    g += gi.double().cpu().numpy()
                    o += r.image
                    cnt += r.image_count
                    edge += r.image_near
        bound = o * (eps + 2.0 ** -23) + cnt * 2.0 ** -33 + edge + 1e-30
        err = np.abs(g - o)
        r = float((err / bound).max())
        worst = max(worst, r)
        _say(f"[fixed image batch {b}] max err/bound {r:.3f}, max rel err "
             f"{float((err / np.maximum(o, 1e-300))[o > 0].max()):.2e}")
        assert np.all(err <= bound)
    _say(f"[fixed image] worst err/bound {worst:.3f}")


def test_fixed_image_estimate_and_mh_reset(R):
    """restore_image_estimate from the integer sums agrees with the batch
    formula on the published float images (float32 rounding of each); the
    MH chain (c_tilde = 0) splats into the integer image too, restore_reset_
    sums clears it, and the image total then equals the chain time."""
    from workloads import pss_render
    from oracle import oracle as O
    wl = pss_render(n_chains=1 << 15, n_steps=128, image=(64, 64), image_batches=8)
    run = R.Run(R.problem_from_workload(wl, flags=R.FLAG_IMAGE_FIXED))
    run.step(wl.n_steps)
    run.drain()
    mean, se = run.image_estimate()
    _sync()
    imgs = run.image.double().cpu().numpy()
    arr = {k: v.cpu().numpy() for k, v in run.arrays().items()}
    run.close()
    tours = np.array([arr["n_done"][lo:hi].astype(np.float64).sum() for lo, hi in O.batch_ranges(wl.n_chains, 8)])
    om, ose = (v.ravel() for v in O.image_batch_estimate(imgs, tours, wl.c_tilde))
    m, s = mean.double().cpu().numpy().ravel(), se.double().cpu().numpy().ravel()
    ok = om > 0
    rel_m = np.abs(m[ok] - om[ok]) / om[ok]
    rel_s = np.abs(s[ok] - ose[ok]) / ose[ok]
    _say(f"[fixed estimate] max rel err mean {rel_m.max():.2e} se {rel_s.max():.2e}")
    assert rel_m.max() < 4 * 2.0 ** -24
    assert rel_s.max() < 1e-4

    mh = R.Run(R.problem_from_workload(wl, c_tilde=0.0, image_batches=1, flags=R.FLAG_IMAGE_FIXED))
    mh.step(40)
    mh.reset_sums()
    mh.step(60)
    _sync()
    tot = float(mh.arrays()["t_done"].sum())
    img = float(mh.image.double().sum())
    mh.close()
    _say(f"[fixed mh image] image total {img:.9g} chain time {tot:.9g}")
    assert abs(img - tot) <= 1e-6 * tot + wl.n_chains * 60 * 2.0 ** -32


def test_fixed_image_flag_validation(R):
    from workloads import gmm_iso_2d, pss_render
    with pytest.raises(R.RestoreError) as e:
        R.Run(R.problem_from_workload(gmm_iso_2d(n_chains=256), flags=R.FLAG_IMAGE_FIXED))
    assert e.value.status == R.E_INVALID_ARG
    wl = pss_render(n_chains=4096, image=(64, 64), image_batches=1)
    with pytest.raises(R.RestoreError) as e:
        R.Run(R.problem_from_workload(wl, flags=R.FLAG_IMAGE_FIXED, tile_px=16))
    assert e.value.status == R.E_UNSUPPORTED
