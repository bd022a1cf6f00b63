"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* brute force: every labeling of tiny lines is enumerated, the Viterbi energies must be
  the true prefix minima (Section 3.2, eqs. viterbi and e(p,u)) and forward + backward -
  cost must be the true min-marginal of the whole line; the sum over the selected paths
  (eq. viterbi) must be the sum of every selected direction's enumerated prefix minima;
* the paper's fast technique (Section 3.3) must equal the full predecessor minimum, also
  at the measured ranges D = 128 and 256;
* special cases with a known answer (lambda = 0, width-1 bands, bands wider than the
  range, constant-disparity warps of i.i.d. noise);
* census invariances and hand-worked census patterns (tests/golden);
* the paper's complexity closed forms (Section 3.4, eqs. Ot-O; tests/golden).
"""
import itertools
import json
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DIRS = [(+1, 0), (-1, 0), (0, +1), (0, -1), (+1, +1), (-1, -1), (-1, +1), (+1, -1)]


def _prefix(x, y, r, w, h):
    """Pixels of the directed line that ends at (x, y), first pixel first."""
    dx, dy = r
    pts = [(x, y)]
    while True:
        px, py = pts[-1][0] - dx, pts[-1][1] - dy
        if not (0 <= px < w and 0 <= py < h):
            break
        pts.append((px, py))
    return pts[::-1]


def _energy(labels, pts, cost, lo, lam, tau):
    e = 0
    for k, ((x, y), d) in enumerate(zip(pts, labels)):
        e += int(cost[y, x, d - (0 if lo is None else lo[y, x])])
        if k:
            a = abs(d - labels[k - 1])
            e += lam * min(a, tau)
    return e


def _band(x, y, lo, ln, cap):
    b0 = 0 if lo is None else int(lo[y, x])
    n = cap if ln is None else int(ln[y, x])
    return range(b0, b0 + n)


def _random_case(rng, w, h, D, banded):
    if banded:
        cap = int(rng.integers(1, D + 1))
        lo = rng.integers(0, D - cap + 1, size=(h, w)).astype(np.int16)
        ln = rng.integers(1, cap + 1, size=(h, w)).astype(np.uint8)
    else:
        cap, lo, ln = D, None, None
    cost = rng.integers(0, 25, size=(h, w, cap)).astype(np.uint8)
    return cost, lo, ln, cap


@pytest.mark.parametrize("banded", [False, True])
@pytest.mark.parametrize("r", range(8))
def test_bruteforce_prefix_minima(orc, r, banded):
    """L_r(p, d) equals the minimum energy over all labelings of the line prefix ending
    at p with label d there: each direction, transition and band rule is checked by
    enumeration."""
    rng = np.random.default_rng(100 + r + 8 * banded)
    for trial in range(6):
        w, h = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        D = int(rng.integers(1, 6))
        lam = int(rng.choice([0, 1, 8]))
        tau = int(rng.choice([1, 2, 4, 9]))
        cost, lo, ln, cap = _random_case(rng, w, h, D, banded)
        for mode in (orc.DEFINITION, orc.FAST):
            L = orc.path(cost, D, r, lam, tau, lo, ln, mode)
            for y in range(h):
                for x in range(w):
                    pts = _prefix(x, y, DIRS[r], w, h)
                    bands = [_band(px, py, lo, ln, cap) for px, py in pts]
                    best = {}
                    for labels in itertools.product(*bands):
                        e = _energy(labels, pts, cost, lo, lam, tau)
                        d = labels[-1]
                        best[d] = min(best.get(d, e), e)
                    b = _band(x, y, lo, ln, cap)
                    for j in range(cap):
                        d = (0 if lo is None else int(lo[y, x])) + j
                        if d in b:
                            assert L[y, x, j] == best[d], (trial, mode, x, y, d)
                        else:
                            assert L[y, x, j] >= orc.INF


@pytest.mark.parametrize("banded", [False, True])
def test_bruteforce_min_marginals(orc, banded):
    """Forward + backward - cost is the exact min-marginal of a whole line (the
    bi-directional merge of Section 3.2 combines exactly these two energies)."""
    rng = np.random.default_rng(7 + banded)
    for trial in range(20):
        n = int(rng.integers(1, 7))
        D = int(rng.integers(1, 6))
        lam = int(rng.choice([0, 1, 8]))
        tau = int(rng.choice([1, 2, 4, 9]))
        cost, lo, ln, cap = _random_case(rng, n, 1, D, banded)
        F = orc.path(cost, D, 0, lam, tau, lo, ln)
        B = orc.path(cost, D, 1, lam, tau, lo, ln)
        pts = [(x, 0) for x in range(n)]
        bands = [_band(x, 0, lo, ln, cap) for x, _ in pts]
        best = {}
        total = None
        for labels in itertools.product(*bands):
            e = _energy(labels, pts, cost, lo, lam, tau)
            total = e if total is None else min(total, e)
            for x, d in enumerate(labels):
                best[(x, d)] = min(best.get((x, d), e), e)
        # the last pixel's minimum forward energy is the global minimum energy
        assert F[0, n - 1][F[0, n - 1] < orc.INF].min() == total
        for (x, d), e in best.items():
            j = d - (0 if lo is None else int(lo[0, x]))
            assert F[0, x, j] + B[0, x, j] - int(cost[0, x, j]) == e


def test_fast_equals_definition(orc):
    """Section 3.3's two-sweep technique gives exactly the full predecessor minimum."""
    rng = np.random.default_rng(11)
    for trial in range(12):
        w, h = int(rng.integers(5, 40)), int(rng.integers(5, 30))
        D = int(rng.integers(1, 48))
        lam = int(rng.integers(0, 12))
        tau = int(rng.integers(1, D + 3))
        cost, lo, ln, cap = _random_case(rng, w, h, D, trial % 2 == 1)
        for r in range(8):
            a = orc.path(cost, D, r, lam, tau, lo, ln, orc.DEFINITION)
            b = orc.path(cost, D, r, lam, tau, lo, ln, orc.FAST)
            np.testing.assert_array_equal(a, b)


def test_lambda_zero_gives_census_wta(orc):
    """With no transition cost every path adds a per-pixel constant to P*C, so WTA of the
    sum is WTA of the cost alone (smallest d on ties)."""
    rng = np.random.default_rng(3)
    left = rng.integers(0, 256, (20, 33), dtype=np.uint8)
    right = rng.integers(0, 256, (20, 33), dtype=np.uint8)
    D = 12
    cv = orc.cost(orc.census(left), orc.census(right), D)
    for P in (1, 2, 4, 8):
        S = orc.aggregate(cv, D, P, 0, 4)
        dl, _, _ = orc.wta_lr(S, D, -1)
        np.testing.assert_array_equal(dl, np.argmin(cv, axis=2))


@pytest.mark.parametrize("d0", [0, 1, 17, 63])
def test_constant_warp_recovered(orc, d0):
    """right(x, y) = left(x + d0, y) on i.i.d. noise: interior pixels get exactly d0 from
    both the left and the right disparity, and pass the LR check."""
    from paper_2001_09678_amd.scene import constant_warp_pair
    D = 64
    left, right = constant_warp_pair(1000 + d0, 160, 48, d0)
    res = orc.pyramid(left, right, D, levels=1, num_paths=4)[0]
    xs = slice(d0 + 8, 160 - 8)
    assert (res.dl[:, xs] == d0).all()
    assert (res.out[:, xs] == d0).all()
    # right disparity: right pixel x_r matches left x_r + d0
    assert (res.dr[:, 8: 160 - 8 - d0] == d0).all()


def test_wide_band_equals_single_scale(orc):
    """A band radius that covers the whole range at every level makes the multi-scale
    result identical to single-scale MPV at the finest level."""
    from paper_2001_09678_amd.scene import make_scene
    sc = make_scene(5, 96, 64, 31, 5)
    ms = orc.pyramid(sc.left, sc.right, 32, levels=3, radius=64, num_paths=8)[-1]
    ss = orc.pyramid(sc.left, sc.right, 32, levels=1, num_paths=8)[-1]
    assert ms.cap == 32
    np.testing.assert_array_equal(ms.dl, ss.dl)
    np.testing.assert_array_equal(ms.out, ss.out)


def test_width_one_band_returns_center(orc):
    from paper_2001_09678_amd.scene import make_scene
    sc = make_scene(6, 64, 48, 31, 4)
    res = orc.pyramid(sc.left, sc.right, 32, levels=2, radius=0, num_paths=4)
    fine = res[-1]
    assert fine.cap == 1
    np.testing.assert_array_equal(fine.dl, fine.lo)


def test_census_golden_patterns(orc):
    blocks = []
    rows = []
    for line in open(os.path.join(GOLDEN, "census_patterns.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("="):
            blocks.append((np.array(rows, dtype=np.uint8), int(line[1:])))
            rows = []
        else:
            rows.append([int(v) for v in line.split()])
    assert len(blocks) == 5
    for img, bits in blocks:
        c = orc.census(img)
        assert bin(int(c[2, 2])).count("1") == bits


def test_census_invariances(orc):
    rng = np.random.default_rng(9)
    img = rng.integers(20, 120, (31, 47), dtype=np.uint8)
    c = orc.census(img)
    assert (c < (1 << 24)).all()
    # a strictly increasing intensity map keeps every comparison
    np.testing.assert_array_equal(orc.census(img + 50), c)
    np.testing.assert_array_equal(orc.census((img.astype(np.int32) * 2).astype(np.uint8)), c)
    # reversing the order flips every strict comparison, ties stay 0: bits(c) + bits(c') = 24 - ties
    inv = orc.census(255 - img)
    assert ((c & inv) == 0).all()
    # Hamming cost is symmetric and bounded by 24; out-of-image candidates cost 24
    other = orc.census(rng.integers(0, 256, (31, 47), dtype=np.uint8))
    cv = orc.cost(c, other, 8)
    assert cv.max() <= 24
    assert (cv[:, 0, 1:] == 24).all()
    cv2 = orc.cost(other, c, 1)
    np.testing.assert_array_equal(cv[:, :, 0], cv2[:, :, 0])


def test_downsample_rounds_half_up(orc):
    img = np.array([[0, 1, 2, 2, 9], [1, 1, 2, 3, 9], [9, 9, 9, 9, 9]], dtype=np.uint8)
    out = orc.downsample(img)
    assert out.shape == (1, 2)
    # (0+1+1+1+2)>>2 = 0.75 -> 1 ; (2+2+2+3+2)>>2 = 2.25 -> 2
    assert out.tolist() == [[1, 2]]
    assert (orc.downsample(np.full((8, 6), 77, np.uint8)) == 77).all()


def test_propagate_hand_example(orc):
    dl = np.array([[0, 3], [10, 15]], dtype=np.int16)
    lo, cap = orc.propagate(dl, 5, 4, 32, 4)
    assert cap == 9
    # center 2*dl, band [clamp(c-4, 0, 32-9), +9)
    expect = np.array([[0, 0, 2, 2, 2], [0, 0, 2, 2, 2], [16, 16, 23, 23, 23], [16, 16, 23, 23, 23]])
    np.testing.assert_array_equal(lo, expect)


def test_wta_lr_hand_example(orc):
    # one row, 4 pixels, D = 3; S chosen by hand
    S = np.array([[[5, 1, 9], [0, 4, 4], [7, 7, 2], [3, 3, 3]]], dtype=np.int64)
    dl, dr, out = orc.wta_lr(S, 3, 1)
    assert dl.tolist() == [[1, 0, 2, 0]]
    # S' rows: [4,0,8] [0,4,4] [5,5,0] [0,0,0]
    # dr(0): d=0 S'(0,0)=4, d=1 S'(1,1)=4, d=2 S'(2,2)=0 -> 2
    # dr(1): S'(1,0)=0, S'(2,1)=5, S'(3,2)=0 -> zero tie, the larger d wins -> 2
    # dr(2): S'(2,0)=5, S'(3,1)=0 -> 1 ; dr(3): S'(3,0)=0 -> 0
    assert dr.tolist() == [[2, 2, 1, 0]]
    # out: x=0 dl=1 -> x-dl<0 -> -1 ; x=1 dl=0 dr(1)=2 -> |0-2|>1 -> -1 ;
    #      x=2 dl=2 dr(0)=2 ok ; x=3 dl=0 dr(3)=0 ok
    assert out.tolist() == [[-1, -1, 2, 0]]


def test_complexity_closed_form(orc):
    """Section 3.4: three layers with d/4 scopes do 0.3281 of single-scale work."""
    g = json.load(open(os.path.join(GOLDEN, "complexity.json")))
    m, n, d = 1280, 720, 128
    sizes = [(m >> 2, n >> 2), (m >> 1, n >> 1), (m, n)]
    dls = orc.level_disparities(d, 3)
    assert dls == [32, 64, 128]
    work = [w * h * (d // 4) for (w, h) in sizes]
    frac = [wk / (m * n * d) for wk in work]
    for got, key in zip(frac, ["layer0", "layer1", "layer2"]):
        assert round(got, 4) == pytest.approx(g[key], abs=1e-4)
    assert round(sum(frac), 4) == pytest.approx(g["three_scale"], abs=1e-4)
    assert sum(frac) == 21 / 64
    # the +/-4 band schedule of the 1280x720, D=128 workload evaluates 12,211,200 nodes
    caps = [32, 9, 9]
    assert sum(w * h * c for (w, h), c in zip(sizes, caps)) == 12_211_200


def _bruteforce_paths(cost, lo, ln, cap, lam, tau):
    """For every direction r, pixel and in-band label: the minimum energy over all labelings
    of the line prefix that ends there (eq. e(p,u) by enumeration)."""
    h, w = cost.shape[:2]
    out = []
    for r in range(8):
        best = {}
        for y in range(h):
            for x in range(w):
                pts = _prefix(x, y, DIRS[r], w, h)
                bands = [_band(px, py, lo, ln, cap) for px, py in pts]
                for labels in itertools.product(*bands):
                    e = _energy(labels, pts, cost, lo, lam, tau)
                    k = (x, y, labels[-1])
                    best[k] = min(best.get(k, e), e)
        out.append(best)
    return out


@pytest.mark.parametrize("banded", [False, True])
def test_bruteforce_path_sum(orc, banded):
    """The sum over the selected Viterbi paths (eq. viterbi): S(p,d) = sum of the
    enumerated prefix minima of every selected direction, for P in {1, 2, 4, 8} and for
    subsets chosen by a path mask; per-path exports equal the enumeration too. A sum that
    drops, repeats or misselects a direction fails here."""
    rng = np.random.default_rng(500 + banded)
    masks = [0, 0b1, 0b10, 0b101, 0b1100, 0b10000000, 0b01010101, 0b11110000, 0b10010110, 0xFF]
    for trial in range(5):
        w, h = int(rng.integers(2, 5)), int(rng.integers(2, 5))
        D = int(rng.integers(2, 5))
        lam = int(rng.choice([1, 3, 8]))
        tau = int(rng.choice([1, 2, 9]))
        cost, lo, ln, cap = _random_case(rng, w, h, D, banded)
        bf = _bruteforce_paths(cost, lo, ln, cap, lam, tau)
        for P in (1, 2, 4, 8):
            for mask in masks:
                sel = [r for r in range(P) if not mask or (mask >> r) & 1]
                S, pp = orc.aggregate(cost, D, P, lam, tau, lo, ln, path_mask=mask, per_path=True)
                if not sel:  # the empty sum
                    assert not S.any() and not pp.any()
                    continue
                for y in range(h):
                    for x in range(w):
                        b0 = 0 if lo is None else int(lo[y, x])
                        band = _band(x, y, lo, ln, cap)
                        for j in range(cap):
                            d = b0 + j
                            if d not in band:
                                assert S[y, x, j] >= orc.INF
                                continue
                            assert S[y, x, j] == sum(bf[r][(x, y, d)] for r in sel), (trial, P, mask, x, y, d)
                            for r in sel:
                                assert pp[r, y, x, j] == bf[r][(x, y, d)]
                # directions outside the selection contribute nothing and are not exported
                for r in range(8):
                    if r not in sel:
                        assert not pp[r].any()


@pytest.mark.parametrize("D", [128, 256])
def test_fast_equals_definition_wide_range(orc, D):
    """The two-sweep technique (Section 3.3) equals the full predecessor minimum at the
    disparity ranges of the measured workloads (D = 128, 256), full range and banded,
    truncated and untruncated."""
    rng = np.random.default_rng(D)
    for trial, tau in enumerate((4, 1, 37, D + 5)):
        w, h = int(rng.integers(6, 12)), int(rng.integers(5, 10))
        lam = int(rng.choice([1, 8, 13]))
        cost, lo, ln, cap = _random_case(rng, w, h, D, trial % 2 == 1)
        for r in range(8):
            a = orc.path(cost, D, r, lam, tau, lo, ln, orc.DEFINITION)
            b = orc.path(cost, D, r, lam, tau, lo, ln, orc.FAST)
            np.testing.assert_array_equal(a, b)
        S_def = orc.aggregate(cost, D, 8, lam, tau, lo, ln, mode=orc.DEFINITION)
        S_fast = orc.aggregate(cost, D, 8, lam, tau, lo, ln, mode=orc.FAST)
        np.testing.assert_array_equal(S_def, S_fast)
