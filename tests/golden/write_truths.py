"""Write the closed-form truths of the synthetic mixture workloads to
tests/golden/truths.json, from the oracle's truth routines only (box
probabilities of Gaussians by Genz's method, the product-of-Gaussians
identity for the integral of p^2).  The benchmark reads this file to score
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
from workloads import gmm_full, gmm_iso_2d  # noqa: E402

PATH = os.path.join(HERE, "truths.json")
WORKLOADS = {"gmm_full_8d": gmm_full, "gmm_iso_2d": gmm_iso_2d}


def compute() -> dict:
    out = {}
    for name, make in WORKLOADS.items():
        wl = make()
        out[name] = {"problem_seed": wl.problem_seed, **truth.truths(wl)}
    return out


if __name__ == "__main__":
    with open(PATH, "w") as f:
        json.dump(compute(), f, indent=1, sort_keys=True)
        f.write("\n")
    print(PATH)
