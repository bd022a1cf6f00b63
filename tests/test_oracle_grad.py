"""Pins of the oracle's gradient-weighted transition (eq. EU: the TV weight lambda * e^-|G|,
with G the left image's intensity difference between consecutive path pixels over sigma,
rounded to an integer) against facts that do not come from the oracle itself.

* brute force: every labeling of tiny lines, each edge weighted by its own gradient;
* reductions: a constant image gives the constant-lambda energies; an edge whose weight
  rounds to 0 decouples the line, so the energies past it are a fresh line's plus the
  minimum reached before it;
* the rounding of the weight cannot depend on the exp implementation: every value of
  lambda * e^(-g/sigma) over the supported range lies at least 6e-8 from a rounding tie;
* the fast technique equals the full predecessor minimum with varying weights, also in the
  layered merge with the occlusion weight.
"""
import itertools
import math

import numpy as np
import pytest

from test_oracle_pins import DIRS, _band, _random_case


def _prefix(x, y, r, w, h):
    dx, dy = r
    pts = [(x, y)]
    while 0 <= pts[-1][0] - dx < w and 0 <= pts[-1][1] - dy < h:
        pts.append((pts[-1][0] - dx, pts[-1][1] - dy))
    return pts[::-1]


def _weight(lam, sigma, g):
    return int(math.floor(lam * math.exp(-g / sigma) + 0.5))


def test_weight_closed_form(orc):
    """g = 0 keeps lambda (e^0 = 1); the weight never exceeds lambda and never increases
    with the gradient; sigma = 0 switches the weighting off."""
    for lam in (0, 1, 8, 57, 255):
        for sigma in (1, 4, 16, 255):
            ws = [orc.grad_weight(lam, sigma, g) for g in range(256)]
            assert ws[0] == lam
            assert all(0 <= a <= lam for a in ws)
            assert all(a >= b for a, b in zip(ws, ws[1:]))
        assert orc.grad_weight(lam, 0, 200) == lam
    assert orc.grad_weight(8, 16, 16) == 3  # 8 / e = 2.94
    assert orc.grad_weight(8, 1, 3) == 0    # 8 / e^3 = 0.40


def test_weight_rounding_has_margin():
    """The weight is decided by rounding lambda * e^(-g/sigma); over lambda <= 255,
    1 <= sigma <= 255 and 0 <= g <= 255 no value lies within 6e-8 of a tie, far beyond the
    last-bit differences of double-precision exp implementations, so any of them (host or
    device) rounds to the same integer."""
    lam = np.arange(0, 256, dtype=np.float64)[:, None, None]
    sig = np.arange(1, 256, dtype=np.float64)[None, :, None]
    g = np.arange(0, 256, dtype=np.float64)[None, None, :]
    v = lam * np.exp(-g / sig)
    assert np.abs(v - np.floor(v) - 0.5).min() > 6e-8


@pytest.mark.parametrize("banded", [False, True])
@pytest.mark.parametrize("r", range(8))
def test_bruteforce_prefix_minima_with_gradient(orc, r, banded):
    rng = np.random.default_rng(500 + r + 8 * banded)
    for trial in range(5):
        w, h = int(rng.integers(1, 5)), int(rng.integers(1, 5))
        D = int(rng.integers(1, 6))
        lam = int(rng.choice([1, 8, 20]))
        tau = int(rng.choice([1, 2, 4, 9]))
        sigma = int(rng.choice([1, 4, 16]))
        cost, lo, ln, cap = _random_case(rng, w, h, D, banded)
        img = rng.integers(0, 256, (h, w), dtype=np.uint8)
        for mode in (orc.DEFINITION, orc.FAST):
            L = orc.path(cost, D, r, lam, tau, lo, ln, mode, img=img, sigma=sigma)
            for y in range(h):
                for x in range(w):
                    pts = _prefix(x, y, DIRS[r], w, h)
                    bands = [_band(px, py, lo, ln, cap) for px, py in pts]
                    best = {}
                    for labels in itertools.product(*bands):
                        e = 0
                        for k, ((px, py), d) in enumerate(zip(pts, labels)):
                            e += int(cost[py, px, d - (0 if lo is None else int(lo[py, px]))])
                            if k:
                                qx, qy = pts[k - 1]
                                wgt = _weight(lam, sigma, abs(int(img[py, px]) - int(img[qy, qx])))
                                e += wgt * min(abs(d - labels[k - 1]), tau)
                        best[labels[-1]] = min(best.get(labels[-1], e), e)
                    b0 = 0 if lo is None else int(lo[y, x])
                    for j in range(cap):
                        if b0 + j in _band(x, y, lo, ln, cap):
                            assert L[y, x, j] == best[b0 + j], (trial, mode, x, y, j)


def test_constant_image_gives_constant_weight(orc):
    rng = np.random.default_rng(51)
    cost, lo, ln, cap = _random_case(rng, 31, 19, 24, True)
    img = np.full((19, 31), 77, np.uint8)
    a = orc.aggregate(cost, 24, 8, 8, 4, lo, ln)
    b = orc.aggregate(cost, 24, 8, 8, 4, lo, ln, img=img, sigma=3)
    np.testing.assert_array_equal(a, b)
    a = orc.layered(cost, 24, 4, 8, 4, lo, ln, occ=True)
    b = orc.layered(cost, 24, 4, 8, 4, lo, ln, occ=True, img=img, sigma=3)
    np.testing.assert_array_equal(a, b)


def test_zero_weight_edge_decouples_the_line(orc):
    """A vertical intensity step whose weight rounds to 0 (8 e^-200): left-to-right energies
    past the step are those of a line starting there plus the minimum reached before it."""
    rng = np.random.default_rng(52)
    h, w, D, x0 = 9, 40, 16, 17
    cost = rng.integers(0, 25, (h, w, D)).astype(np.uint8)
    img = np.zeros((h, w), np.uint8)
    img[:, x0:] = 200
    full = orc.path(cost, D, 0, 8, 4, img=img, sigma=1)
    fresh = orc.path(np.ascontiguousarray(cost[:, x0:]), D, 0, 8, 4)
    offset = full[:, x0 - 1].min(axis=1)[:, None, None]
    np.testing.assert_array_equal(full[:, x0:], fresh + offset)
    # without the step the line stays coupled
    coupled = orc.path(cost, D, 0, 8, 4, img=np.zeros((h, w), np.uint8), sigma=1)
    assert not np.array_equal(coupled[:, x0:], fresh + coupled[:, x0 - 1].min(axis=1)[:, None, None])


def test_fast_equals_definition_with_gradient(orc):
    rng = np.random.default_rng(53)
    for trial in range(8):
        w, h = int(rng.integers(5, 30)), int(rng.integers(5, 25))
        D = int(rng.integers(1, 40))
        lam = int(rng.integers(0, 12))
        tau = int(rng.integers(1, D + 3))
        sigma = int(rng.choice([1, 5, 30]))
        cost, lo, ln, cap = _random_case(rng, w, h, D, trial % 2 == 1)
        img = rng.integers(0, 256, (h, w), dtype=np.uint8)
        for r in range(8):
            a = orc.path(cost, D, r, lam, tau, lo, ln, orc.DEFINITION, img=img, sigma=sigma)
            b = orc.path(cost, D, r, lam, tau, lo, ln, orc.FAST, img=img, sigma=sigma)
            np.testing.assert_array_equal(a, b)
        for occ in (False, True):
            a = orc.layered(cost, D, 4, lam, tau, lo, ln, occ=occ, mode=orc.DEFINITION, img=img, sigma=sigma)
            b = orc.layered(cost, D, 4, lam, tau, lo, ln, occ=occ, mode=orc.FAST, img=img, sigma=sigma)
            np.testing.assert_array_equal(a, b)
