"""Pins of the oracle's tile-stratified restore runs -- no GPU.

Tile-stratified restore cuts the image into tiles and runs each tile as its
own restore problem: target p restricted to the tile, mu uniform on it, the
killing constant c_tilde A_t (A_t the tile's share of the box) so that the
killing rate stays c_tilde / p.  By Sec. 6.3 applied per tile, tile t's
tour ratio estimates its own mass int_tile p, and the tiles add up to
p_lambda.  Pinned on the 2-D mixture, where every tile's mass is a product
of erf differences (closed form, independent of the oracle).
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import truth
from tests import helpers as H
from workloads import gmm_iso_2d

IMG = (64, 64)
TILE = 16


def _problem(wl, **kw):
    return O.Problem(wl, image=IMG, tile_px=TILE, **kw)


def test_tile_geometry_and_chain_map(oracle_lib):
    wl = gmm_iso_2d(n_chains=1000)
    prob = O.Problem(wl, image=(50, 37), tile_px=16)
    rng, area = O.tiles(prob)
    assert len(rng) == 4 * 3 and abs(area.sum() - 1.0) < 1e-15
    assert rng[3] == (48, 50, 0, 16) and rng[-1] == (48, 50, 32, 37)
    tid = O.tile_of_chain(prob, np.arange(1000))
    assert tid[0] == 0 and tid[-1] == 11 and np.all(np.diff(tid) >= 0)
    counts = np.bincount(tid)
    assert counts.min() >= 83 and counts.max() <= 84


def test_initial_states_lie_in_their_tiles(oracle_lib):
    wl = gmm_iso_2d(n_chains=4096)
    prob = _problem(wl)
    st = O.init_states(prob, np.arange(wl.n_chains))
    rng, _ = O.tiles(prob)
    tid = O.tile_of_chain(prob, np.arange(wl.n_chains))
    px = np.floor(st.x[:, 0] * IMG[0]).astype(int)
    py = np.floor(st.x[:, 1] * IMG[1]).astype(int)
    for c in range(wl.n_chains):
        a0, a1, b0, b1 = rng[tid[c]]
        assert a0 <= px[c] < a1 and b0 <= py[c] < b1
    # uniform inside the tile: the mean offset is half the tile
    off = st.x[:, 0] * IMG[0] - np.array([rng[t][0] for t in tid])
    assert abs(off.mean() - TILE / 2) < 0.2


def test_chains_stay_in_their_tile(oracle_lib):
    """A tile's chains splat only into the tile's pixels."""
    wl = gmm_iso_2d(n_chains=4096, n_steps=300)
    prob = _problem(wl)
    tid = O.tile_of_chain(prob, np.arange(wl.n_chains))
    rng, _ = O.tiles(prob)
    for t in (5, 6, 9):
        lo, hi = np.flatnonzero(tid == t)[[0, -1]]
        r = O.run(prob, int(lo), int(hi) + 1)
        a0, a1, b0, b1 = rng[t]
        inside = r.image[b0:b1, a0:a1].sum()
        outside = r.image.copy()
        outside[b0:b1, a0:a1] = 0.0
        assert inside > 0 and not outside.any()
        assert abs(inside - r.t_done.sum()) < 1e-9 * inside


def test_stratified_estimates_match_tile_masses_and_truth(oracle_lib):
    """Every tile's p_lambda estimate against its erf mass (|z| < 4), the
    stratified totals within 3 SE of the erf truths, and the z-scores of
    the 16 tiles spread like a standard normal."""
    wl = gmm_iso_2d()
    prob = _problem(wl)
    r = O.run(prob, 0, wl.n_chains)
    est = O.estimate_tiles(prob, r)
    assert est["tours_censored"] == 0
    masses = H.iso_cell_masses(wl, np.linspace(0, 1, IMG[0] // TILE + 1))
    z = []
    for tt in est["tiles"]:
        t = tt["tile"]
        tx, ty = t % (IMG[0] // TILE), t // (IMG[0] // TILE)
        m = masses[tx, ty]
        if m > 1e-3:
            z.append((tt["p_lambda"] - m) / tt["p_lambda_se"])
    z = np.array(z)
    assert len(z) >= 8 and np.all(np.abs(z) < 4), z
    assert abs(z.mean()) < 4 / np.sqrt(len(z)) and 0.4 < z.std() < 1.8
    tr = truth.truths(wl)
    for key in ("p_lambda", "lam_pf", "pi_f"):
        assert abs(est[key] - tr[key]) < 3 * est[key + "_se"], key
    # the image estimate sums to the p_lambda estimate
    img = O.image_estimate_tiles(prob, r)
    assert abs(img.sum() - est["p_lambda"]) < 1e-9 * est["p_lambda"]
