"""Pins of the oracle's SSIM data term (Section 3.2, eqs. components and ssim, with the cited
structural-similarity work's constants K1 = 0.01, K2 = 0.03, L = 255, C3 = C2/2, alpha = beta
= gamma = 1, 5x5 box patches, cost (1 - SSIM) * 24 / 2 rounded half up) against facts that do
not come from the oracle: identical patches cost 0, the index is symmetric, hand-computed
exact ratios of constant patches, an independent float64 evaluation of the three separate
components (with the square roots the oracle's identity removes), a monotone luminance
response, contrast inversion, and exact zeros at the true disparity of a constant warp."""
from fractions import Fraction

import numpy as np
import pytest


def _float_ssim(psi, phi):
    """The three components of the cited work in float64, each from its own definition."""
    x = psi.astype(np.float64).ravel()
    y = phi.astype(np.float64).ravel()
    C1, C2 = (0.01 * 255) ** 2, (0.03 * 255) ** 2
    C3 = C2 / 2
    mx, my = x.mean(), y.mean()
    vx, vy = ((x - mx) ** 2).mean(), ((y - my) ** 2).mean()
    cxy = ((x - mx) * (y - my)).mean()
    sx, sy = np.sqrt(vx), np.sqrt(vy)
    l = (2 * mx * my + C1) / (mx ** 2 + my ** 2 + C1)
    c = (2 * sx * sy + C2) / (vx + vy + C2)
    s = (cxy + C3) / (sx * sy + C3)
    return l * c * s


def test_identical_patches_cost_zero(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        p = rng.integers(0, 256, 25, dtype=np.uint8)
        num, den = orc.ssim_ratio(p, p)
        assert num == den
        assert orc.ssim_patch_cost(p, p) == 0


def test_symmetry(orc):
    rng = np.random.default_rng(2)
    for _ in range(200):
        a = rng.integers(0, 256, 25, dtype=np.uint8)
        b = rng.integers(0, 256, 25, dtype=np.uint8)
        assert orc.ssim_ratio(a, b) == orc.ssim_ratio(b, a)
        assert orc.ssim_patch_cost(a, b) == orc.ssim_patch_cost(b, a)


@pytest.mark.parametrize("u,v,expect_cost", [(100, 110, 0), (0, 255, 12), (40, 200, 7), (128, 128, 0)])
def test_constant_patches_hand_computed(orc, u, v, expect_cost):
    """Flat patches have no variance, so c = s = 1 and SSIM = l = (2uv + C1) / (u^2 + v^2 + C1)
    with C1 = 6.5025. By hand: 100 vs 110: l = 22006.5025 / 22106.5025 = 0.99548, cost
    12 (1 - l) = 0.054 -> 0; 0 vs 255: l = 6.5025 / 65031.5025, cost 11.9988 -> 12;
    40 vs 200: l = 16006.5025 / 41606.5025 = 0.38471, cost 7.383 -> 7."""
    a = np.full(25, u, np.uint8)
    b = np.full(25, v, np.uint8)
    num, den = orc.ssim_ratio(a, b)
    C1 = Fraction(65025, 10000)
    assert Fraction(num, den) == (2 * u * v + C1) / (u * u + v * v + C1)
    assert orc.ssim_patch_cost(a, b) == expect_cost


def test_agrees_with_three_component_float64(orc):
    """On random and structured patch pairs the exact ratio equals the float64 product of the
    three separately computed components (square roots included) to rounding error, and the
    quantised cost equals the float64 one wherever that is not within 1e-9 of a rounding tie."""
    rng = np.random.default_rng(3)
    cases = []
    for _ in range(400):
        a = rng.integers(0, 256, 25, dtype=np.uint8)
        kind = rng.integers(0, 4)
        if kind == 0:
            b = rng.integers(0, 256, 25, dtype=np.uint8)
        elif kind == 1:  # noisy copy
            b = np.clip(a.astype(int) + rng.integers(-12, 13, 25), 0, 255).astype(np.uint8)
        elif kind == 2:  # contrast and brightness change
            b = np.clip(a.astype(int) // 2 + 60, 0, 255).astype(np.uint8)
        else:  # low-texture patches
            a = rng.integers(100, 104, 25, dtype=np.uint8)
            b = rng.integers(100, 106, 25, dtype=np.uint8)
        cases.append((a, b))
    for a, b in cases:
        num, den = orc.ssim_ratio(a, b)
        ref = _float_ssim(a, b)
        assert abs(num / den - ref) < 1e-12, (a, b)
        x = 12.0 * (1.0 - ref)
        if abs(x - np.floor(x) - 0.5) > 1e-9:
            assert orc.ssim_patch_cost(a, b) == int(np.floor(x + 0.5))


def test_monotone_luminance_response(orc):
    """Two flat patches: the cost never decreases as their intensities move apart."""
    a = np.full(25, 128, np.uint8)
    prev = 0
    for t in range(0, 128):
        c = orc.ssim_patch_cost(a, np.full(25, 128 + t, np.uint8))
        assert c >= prev
        prev = c
    assert prev > 0


def test_contrast_inversion(orc):
    """A patch against its photographic negative is anti-correlated: SSIM < 0, cost > 12."""
    rng = np.random.default_rng(4)
    for _ in range(50):
        a = rng.integers(60, 196, 25, dtype=np.uint8)
        num, den = orc.ssim_ratio(a, 255 - a)
        assert num < 0 < den
        assert orc.ssim_patch_cost(a, 255 - a) > 12


@pytest.mark.parametrize("d0", [0, 3, 17])
def test_volume_constant_warp(orc, d0):
    """right(x, y) = left(x + d0, y): every pixel whose two patches need no clamping against
    each other costs 0 at d0; candidates with x - d < 0 cost 24; bands pick the same slots
    as the full range and fill the rest with 0xFF."""
    from paper_2001_09678_amd.scene import constant_warp_pair
    W, H, D = 64, 20, 24
    left, right = constant_warp_pair(77 + d0, W, H, d0)
    cv = orc.ssim_cost(left, right, D)
    assert cv.shape == (H, W, D) and cv.max() <= 24
    assert (cv[:, d0 + 2: W - 2, d0] == 0).all()
    for x in range(W):
        assert (cv[:, x, x + 1:] == 24).all()
    # lambda = 0 WTA recovers d0 where the patches are unique (i.i.d. noise)
    assert (np.argmin(cv[:, D + 2: W - 2], axis=2) == d0).all()
    rng = np.random.default_rng(d0)
    cap = 7
    lo = rng.integers(0, D - cap + 1, size=(H, W)).astype(np.int16)
    ln = rng.integers(1, cap + 1, size=(H, W)).astype(np.uint8)
    cb = orc.ssim_cost(left, right, D, lo, ln, cap)
    for y in range(H):
        for x in range(W):
            for j in range(cap):
                want = cv[y, x, lo[y, x] + j] if j < ln[y, x] else 255
                assert cb[y, x, j] == want


def test_pyramid_with_ssim_recovers_constant_warp(orc):
    """Single-scale MPV over the SSIM data term recovers a constant disparity of i.i.d.
    noise exactly away from the borders (left, right and LR-checked maps)."""
    from paper_2001_09678_amd.scene import constant_warp_pair
    d0 = 9
    left, right = constant_warp_pair(5, 96, 32, d0)
    res = orc.pyramid(left, right, 32, levels=1, num_paths=4, data_term="ssim")[0]
    xs = slice(d0 + 8, 96 - 8)
    assert (res.dl[:, xs] == d0).all()
    assert (res.out[:, xs] == d0).all()
