"""Write the closed-form truths of the synthetic workloads to
tests/golden/truths.json, from the oracle's truth routines only (box
probabilities of Gaussians by Genz's method, the product-of-Gaussians
identity for the integral of p^2; for the rendering-shaped integrand the
per-pixel integrals, closed form plus Gauss-Legendre for the lobe, summed
over 8 x 8-pixel tiles).  The benchmark reads this file to score
estimates; tests/test_oracle_pins.py checks it against a fresh computation.

    python tests/golden/write_truths.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import truth  # noqa: E402
from workloads import batched_family, batched_uneven, gmm_full, gmm_iso_2d, pss_render  # noqa: E402

PATH = os.path.join(HERE, "truths.json")
WORKLOADS = {"gmm_full_8d": gmm_full, "gmm_iso_2d": gmm_iso_2d}
PSS_TILE = 8   # the image truth is stored as sums over 8 x 8-pixel tiles


def _uneven_p_lambda(i: int) -> float:
    return truth.gmm_full_p_lambda(batched_uneven()[i])


def compute(uneven_targets=None) -> dict:
    """All stored truths; `uneven_targets` limits the 256 batched targets
    to the given indices (the pins check a sample: the full set takes
    minutes of Genz integration)."""
    out = {}
    for name, make in WORKLOADS.items():
        wl = make()
        out[name] = {"problem_seed": wl.problem_seed, **truth.truths(wl)}
    wl = pss_render()
    img = truth.pss_pixel_truth(wl, gl_order=8)
    h, w = img.shape
    tiles = img.reshape(h // PSS_TILE, PSS_TILE, w // PSS_TILE, PSS_TILE).sum(axis=(1, 3))
    out["pss_render_12d"] = {"problem_seed": wl.problem_seed, "p_lambda": float(img.sum()),
                             "image": [w, h], "tile": PSS_TILE,
                             "tiles": [[float(v) for v in row] for row in tiles]}
    fam = batched_family()
    out["batched_family_8d"] = {"problem_seed": fam[0].problem_seed,
                                "p_lambda": [truth.gmm_full_p_lambda(t) for t in fam]}
    # the 256 batched targets (d up to 16, K up to 32): p_lambda only,
    # the box probabilities of their components by Genz's method
    from multiprocessing import Pool
    uneven = batched_uneven()
    idx = range(len(uneven)) if uneven_targets is None else list(uneven_targets)
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        pl = pool.map(_uneven_p_lambda, idx)
    out["batched_uneven"] = {"problem_seed": uneven[0].problem_seed, "p_lambda": [float(v) for v in pl]}
    return out


if __name__ == "__main__":
    with open(PATH, "w") as f:
        json.dump(compute(), f, indent=1, sort_keys=True)
        f.write("\n")
    print(PATH)
