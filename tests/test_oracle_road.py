"""Pins of the road-profile oracle (Section 3.5: the v-disparity image of eq. disp_map, the
u-disparity image of eq. hy and the road Viterbi of eqs. P_hat and e) against facts that
do not come from it.

* v-disparity: a hand-counted example and the invariants of a histogram (each row's
  counts add up to its valid pixels; invalid and out-of-range disparities are ignored);
* u-disparity (eq. hy): a hand-counted example, each column's counts add up to its valid
  pixels, and it equals the v-disparity image of the transposed map;
* road Viterbi: enumeration of every admissible path (0 < row step < eta) on tiny
  histograms gives the same maximum energy, and the returned profile is admissible and
  reaches it; closed forms: a dominant straight line is recovered exactly, a ground plane
  whose disparity grows linearly below the horizon over the whole range is followed row
  for row, and a histogram too short for D-1 row steps has no profile.
"""
import itertools

import numpy as np
import pytest


@pytest.fixture(scope="module")
def road():
    from oracle import road as r
    return r


def test_vdisparity_hand_example(road):
    disp = np.array([[0, 1, 1, -1],
                     [2, 2, 2, 2],
                     [5, 0, -1, 3]], np.int16)
    h = road.vdisparity(disp, 4)
    assert h.shape == (4, 3) and h.dtype == np.uint32
    np.testing.assert_array_equal(h[:, 0], [1, 2, 0, 0])
    np.testing.assert_array_equal(h[:, 1], [0, 0, 4, 0])
    np.testing.assert_array_equal(h[:, 2], [1, 0, 0, 1])  # 5 >= D and -1 are not counted


def test_vdisparity_invariants(road):
    rng = np.random.default_rng(60)
    disp = rng.integers(-1, 40, (37, 53)).astype(np.int16)
    h = road.vdisparity(disp, 32)
    valid = (disp >= 0) & (disp < 32)
    np.testing.assert_array_equal(h.sum(axis=0), valid.sum(axis=1))
    assert h.sum() == valid.sum()
    for i in (0, 7, 31):
        np.testing.assert_array_equal(h[i], (disp == i).sum(axis=1))


def _admissible(path, eta, H):
    p = [int(v) for v in path]
    return all(0 <= v < H for v in p) and all(0 < b - a < eta for a, b in zip(p, p[1:]))


@pytest.mark.parametrize("eta", [2, 3, 4])
def test_road_bruteforce(road, eta):
    rng = np.random.default_rng(61 + eta)
    for trial in range(12):
        D, H = int(rng.integers(1, 5)), int(rng.integers(1, 9))
        hist = rng.integers(0, 6, (D, H)).astype(np.uint32)
        best = None
        for path in itertools.product(range(H), repeat=D):
            if _admissible(path, eta, H):
                e = sum(int(hist[i, j]) for i, j in enumerate(path))
                best = e if best is None else max(best, e)
        path, energy = road.road(hist, eta)
        if best is None:
            assert energy == -1 and (path == -1).all()
        else:
            assert energy == best
            assert _admissible(path, eta, H)
            assert sum(int(hist[i, j]) for i, j in enumerate(path)) == best


def test_road_recovers_a_dominant_line(road):
    rng = np.random.default_rng(62)
    D, H, eta = 48, 200, 6
    hist = rng.integers(0, 3, (D, H)).astype(np.uint32)
    line = 20 + 3 * np.arange(D)
    hist[np.arange(D), line] += 50
    path, energy = road.road(hist, eta)
    np.testing.assert_array_equal(path, line)
    assert energy == int(hist[np.arange(D), line].sum())


def test_road_follows_a_ground_plane(road):
    """A ground plane whose disparity grows linearly from 0 at the horizon yh to D-1 at the
    bottom row, invalid above: every disparity owns one or more consecutive rows and the
    profile lies on one of them at every disparity. (A profile spans every disparity with
    at least one row per step, so a ramp that ends below D-1 cannot be followed to its end.)"""
    W, H, D = 64, 240, 64
    yh = H // 2
    y = np.arange(H)
    d = np.where(y >= yh, np.floor((D - 1) * (y - yh) / (H - 1 - yh) + 0.5), -1).astype(np.int16)
    disp = np.repeat(d[:, None], W, axis=1)
    path, energy = road.road(road.vdisparity(disp, D), eta=8)
    owned = 0
    for i in range(D):
        rows = np.nonzero(d == i)[0]
        if len(rows):
            owned += 1
            assert rows.min() <= path[i] <= rows.max(), (i, path[i], rows)
    assert owned == D


def test_road_unreachable(road):
    path, energy = road.road(np.ones((6, 4), np.uint32), eta=3)  # needs 5 row steps in 4 rows
    assert energy == -1 and (path == -1).all()


def test_udisparity_hand_example_and_invariants(road):
    disp = np.array([[0, 1, 1, -1],
                     [2, 2, 1, 2],
                     [5, 0, -1, 3]], np.int16)
    h = road.udisparity(disp, 4)
    assert h.shape == (4, 4) and h.dtype == np.uint32
    np.testing.assert_array_equal(h[:, 0], [1, 0, 1, 0])  # 5 >= D is not counted
    np.testing.assert_array_equal(h[:, 1], [1, 1, 1, 0])
    np.testing.assert_array_equal(h[:, 2], [0, 2, 0, 0])
    np.testing.assert_array_equal(h[:, 3], [0, 0, 1, 1])
    rng = np.random.default_rng(63)
    disp = rng.integers(-1, 40, (29, 47)).astype(np.int16)
    h = road.udisparity(disp, 32)
    valid = (disp >= 0) & (disp < 32)
    np.testing.assert_array_equal(h.sum(axis=0), valid.sum(axis=0))
    # the transpose of the map has the v-disparity image of this map's u-disparity
    np.testing.assert_array_equal(h, road.vdisparity(disp.T.copy(), 32))
