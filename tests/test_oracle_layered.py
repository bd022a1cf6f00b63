"""Pins of the oracle's layered path merge (Section 3.2: hierarchical merging of the
bi-directional paths, Table alg) against facts that do not come from the oracle itself.

* brute force: on tiny images every layer is recomputed from its own input (the cost for
  the first layer, the oracle's previous layer for the others) by enumerating every
  labeling of every line prefix and suffix, with the min merge for the horizontal layer,
  the floor mean for the others and the doubled upward weight of the occlusion strategy;
* closed forms: lambda = 0 leaves every layer equal to the cost minus its pixel minimum;
  single-row and single-column images reduce to one horizontal or vertical layer;
* invariants: a per-pixel constant added to a layer's input changes nothing (so the merged
  energies need no normalisation before they seed the next layer), and layer k's merged
  energies stay within 24 + (k+1) * lambda * tau for census costs (so they fit a byte);
* the paper's fast technique (Section 3.3) with the asymmetric weight equals the full
  predecessor minimum;
* constant-disparity warps of i.i.d. noise are recovered exactly.
"""
import itertools

import numpy as np
import pytest

from test_oracle_pins import DIRS, _band, _random_case


def _line_prefix(x, y, r, w, h):
    dx, dy = r
    pts = [(x, y)]
    while 0 <= pts[-1][0] - dx < w and 0 <= pts[-1][1] - dy < h:
        pts.append((pts[-1][0] - dx, pts[-1][1] - dy))
    return pts[::-1]


def _energy(labels, pts, data, lo, lam, tau, up):
    e = 0
    for k, ((x, y), d) in enumerate(zip(pts, labels)):
        e += int(data[y, x, d - (0 if lo is None else int(lo[y, x]))])
        if k:
            dp = labels[k - 1]
            e += (up if d > dp else 1) * lam * min(abs(d - dp), tau)
    return e


def _brute_direction(data, lo, ln, cap, r, lam, tau, up):
    """Minimum energy over all labelings of the line prefix ending at p with d there."""
    h, w, _ = data.shape
    out = {}
    for y in range(h):
        for x in range(w):
            pts = _line_prefix(x, y, DIRS[r], w, h)
            bands = [_band(px, py, lo, ln, cap) for px, py in pts]
            for labels in itertools.product(*bands):
                e = _energy(labels, pts, data, lo, lam, tau, up)
                key = (x, y, labels[-1])
                out[key] = min(out.get(key, e), e)
    return out


def _brute_layer(data, lo, ln, cap, k, lam, tau, occ):
    h, w, _ = data.shape
    F = _brute_direction(data, lo, ln, cap, 2 * k, lam, tau, 2 if (occ and k == 0) else 1)
    B = _brute_direction(data, lo, ln, cap, 2 * k + 1, lam, tau, 1)
    M = {}
    for y in range(h):
        for x in range(w):
            ds = list(_band(x, y, lo, ln, cap))
            fm = min(F[(x, y, d)] for d in ds)
            bm = min(B[(x, y, d)] for d in ds)
            for d in ds:
                f, b = F[(x, y, d)] - fm, B[(x, y, d)] - bm
                M[(x, y, d)] = min(f, b) if k == 0 else (f + b) // 2
    return M


@pytest.mark.parametrize("occ", [False, True])
@pytest.mark.parametrize("banded", [False, True])
def test_bruteforce_every_layer(orc, banded, occ):
    rng = np.random.default_rng(300 + 2 * banded + occ)
    for trial in range(5):
        w, h = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        D = int(rng.integers(1, 5))
        lam = int(rng.choice([0, 1, 3, 8]))
        tau = int(rng.choice([1, 2, 4, 9]))
        cost, lo, ln, cap = _random_case(rng, w, h, D, banded)
        for mode in (orc.DEFINITION, orc.FAST):
            M, per = orc.layered(cost, D, 4, lam, tau, lo, ln, occ=occ, mode=mode, per_layer=True)
            np.testing.assert_array_equal(M, per[-1])
            for k in range(4):
                data = cost.astype(np.int64) if k == 0 else per[k - 1]
                ref = _brute_layer(data, lo, ln, cap, k, lam, tau, occ)
                for y in range(h):
                    for x in range(w):
                        b0 = 0 if lo is None else int(lo[y, x])
                        ds = _band(x, y, lo, ln, cap)
                        for j in range(cap):
                            if b0 + j in ds:
                                assert per[k, y, x, j] == ref[(x, y, b0 + j)], (trial, mode, k, x, y, j)
                            else:
                                assert per[k, y, x, j] >= orc.INF


def test_lambda_zero_is_normalised_cost(orc):
    """With no transition weight each pass adds a per-pixel constant to the data term, so
    every layer's merge is the cost minus the pixel's minimum cost."""
    rng = np.random.default_rng(31)
    for banded in (False, True):
        cost, lo, ln, cap = _random_case(rng, 23, 17, 20, banded)
        M, per = orc.layered(cost, 20, 4, 0, 4, lo, ln, per_layer=True)
        bn = np.full(cost.shape[:2], cap) if ln is None else ln.astype(int)
        inb = np.arange(cap)[None, None, :] < bn[:, :, None]
        c = np.where(inb, cost.astype(np.int64), np.int64(1) << 40)
        norm = c - c.min(axis=2, keepdims=True)
        for k in range(4):
            np.testing.assert_array_equal(per[k][inb], norm[inb])


def test_single_row_and_column_reduce_to_one_layer(orc):
    """On a single row every non-horizontal line is one pixel, so each later layer only
    subtracts the pixel minimum from the horizontal merge; on a single column the same
    holds for the vertical merge (the horizontal layer merely normalises the cost)."""
    rng = np.random.default_rng(32)
    cost = rng.integers(0, 25, (1, 29, 9)).astype(np.uint8)
    M1 = orc.layered(cost, 9, 1, 8, 4)
    M4 = orc.layered(cost, 9, 4, 8, 4)
    np.testing.assert_array_equal(M4, M1 - M1.min(axis=2, keepdims=True))
    cost = rng.integers(0, 25, (31, 1, 9)).astype(np.uint8)
    M2 = orc.layered(cost, 9, 2, 8, 4)
    M4 = orc.layered(cost, 9, 4, 8, 4)
    np.testing.assert_array_equal(M4, M2 - M2.min(axis=2, keepdims=True))


def test_per_pixel_offset_of_the_data_term_changes_nothing(orc):
    """Adding c(p) to every disparity of pixel p shifts each pass's energies at p by a
    constant, which the per-pixel minimum removes: every layer's merge is unchanged."""
    rng = np.random.default_rng(33)
    cost = rng.integers(0, 25, (19, 27, 16)).astype(np.uint8)
    off = rng.integers(0, 200, (19, 27, 1)).astype(np.uint8)
    a = orc.layered(cost, 16, 4, 8, 4, per_layer=True)[1]
    b = orc.layered(cost + off, 16, 4, 8, 4, per_layer=True)[1]
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("occ", [False, True])
def test_merged_energies_fit_a_byte(orc, occ):
    """Layer k's merged energies lie in [0, 24 + (k+1) * lambda * min(tau, D-1)] for census
    costs: a pass's energy at p exceeds its pixel minimum by at most the range of the data
    term plus lambda * tau, and both merges keep that bound (the doubled weight only enters
    the first layer, whose min merge takes the other pass where it is larger)."""
    from paper_2001_09678_amd.scene import make_scene
    sc = make_scene(34, 96, 64, 47, 6)
    D, lam, tau = 48, 8, 4
    cv = orc.cost(orc.census(sc.left), orc.census(sc.right), D)
    _, per = orc.layered(cv, D, 4, lam, tau, occ=occ, per_layer=True)
    for k in range(4):
        assert per[k].min() >= 0
        assert per[k].max() <= 24 + (k + 1) * lam * tau, (k, per[k].max())


def test_fast_equals_definition_with_occlusion_weight(orc):
    rng = np.random.default_rng(35)
    for trial in range(8):
        w, h = int(rng.integers(5, 30)), int(rng.integers(5, 25))
        D = int(rng.integers(1, 40))
        lam = int(rng.integers(0, 12))
        tau = int(rng.integers(1, D + 3))
        cost, lo, ln, cap = _random_case(rng, w, h, D, trial % 2 == 1)
        for occ in (False, True):
            a = orc.layered(cost, D, 4, lam, tau, lo, ln, occ=occ, mode=orc.DEFINITION, per_layer=True)[1]
            b = orc.layered(cost, D, 4, lam, tau, lo, ln, occ=occ, mode=orc.FAST, per_layer=True)[1]
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("occ", [False, True])
@pytest.mark.parametrize("d0", [0, 5, 30])
def test_constant_warp_recovered(orc, d0, occ):
    from paper_2001_09678_amd.scene import constant_warp_pair
    D = 64
    left, right = constant_warp_pair(2000 + d0, 128, 40, d0)
    res = orc.pyramid(left, right, D, levels=1, num_paths=8, merge="layered", occ=occ)[0]
    xs = slice(d0 + 8, 128 - 8)
    assert (res.dl[:, xs] == d0).all()
    assert (res.out[:, xs] == d0).all()
