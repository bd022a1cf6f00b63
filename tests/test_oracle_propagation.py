"""Pins of the oracle's version of the paper's propagation (Section 3.4: block modes at the
intermediate layers, linear interpolation at the last layer, d/4-wide scopes), against
facts that do not come from the oracle: constant maps, linear ramps (which linear
interpolation reproduces exactly), modes counted independently, a hand-worked example and
the reduction to single-scale matching when the band covers the whole range."""
from collections import Counter

import numpy as np
import pytest


def _clamp(v, lo, hi):
    return max(lo, min(hi, v))


@pytest.mark.parametrize("R,Dl", [(4, 64), (16, 128), (0, 32)])
def test_constant_map(orc, R, Dl):
    dl = np.full((9, 13), 11, np.int16)
    cap = min(2 * R + 1, Dl)
    expect = _clamp(22 - R, 0, Dl - cap)
    for lo, c in (orc.propagate_block(dl, 26, 18, Dl, R, 8), orc.propagate_block(dl, 27, 19, Dl, R, 4),
                  orc.propagate_interp(dl, 26, 18, Dl, R), orc.propagate_interp(dl, 27, 19, Dl, R)):
        assert c == cap
        assert (lo == expect).all()


@pytest.mark.parametrize("a,b", [(1, 0), (0, 1), (2, 3), (3, 1)])
def test_linear_ramp_interpolates_exactly(orc, a, b):
    """A coarse map linear in (i, j) becomes the fine ramp a*x + b*y: the samples carry
    twice the coarse value and every interpolated pixel lies on the same plane."""
    Wc, Hc = 12, 9
    j, i = np.mgrid[0:Hc, 0:Wc]
    dl = (a * i + b * j).astype(np.int16)
    W, H = 2 * Wc, 2 * Hc
    lo, cap = orc.propagate_interp(dl, W, H, 256, 0)
    assert cap == 1
    y, x = np.mgrid[0:H, 0:W]
    inner = (x < W - 1) & (y < H - 1)  # the last fine row/column has no sample beyond it
    np.testing.assert_array_equal(lo[inner], (a * x + b * y)[inner])
    # past the last sample column / row the interpolation holds the last samples
    np.testing.assert_array_equal(lo[:, -1], lo[:, -2])
    np.testing.assert_array_equal(lo[-1, :], lo[-2, :])


def test_interp_midpoints_and_rounding(orc):
    """Hand-worked: coarse 0, 3 / 5, 8 give the samples 0, 6 / 10, 16 at the even fine
    pixels; the pixels between them take the means."""
    dl = np.array([[0, 3], [5, 8]], np.int16)
    lo, _ = orc.propagate_interp(dl, 4, 4, 64, 0)
    # samples: (0,0)=0 (2,0)=6 (0,2)=10 (2,2)=16; midpoints: (1,0)=3 (0,1)=5 (1,1)=(0+6+10+16+2)>>2=8
    # (3,*) and (*,3) clamp to the last sample column/row
    expect = np.array([[0, 3, 6, 6],
                       [5, 8, 11, 11],
                       [10, 13, 16, 16],
                       [10, 13, 16, 16]])
    np.testing.assert_array_equal(lo, expect)
    # rounding of the four-sample centre: 0, 2, 2, 2 doubled -> (0+4+4+4+2)>>2 = 3 (3.0 exactly);
    # 0, 0, 0, 1 doubled -> (2+2)>>2 = 1 (0.5 rounds half up)
    lo, _ = orc.propagate_interp(np.array([[0, 0], [0, 1]], np.int16), 3, 3, 64, 0)
    assert lo[1, 1] == 1
    lo, _ = orc.propagate_interp(np.array([[0, 2], [2, 2]], np.int16), 3, 3, 64, 0)
    assert lo[1, 1] == 3


def _block_mode_reference(dl, W, H, block):
    """Mode of twice the parents' values of each block (most frequent, smallest on ties),
    counted with a Counter over the distinct parents."""
    Hc, Wc = dl.shape
    out = np.empty((H, W), np.int64)
    for by in range(0, H, block):
        for bx in range(0, W, block):
            parents = {(min(x // 2, Wc - 1), min(y // 2, Hc - 1))
                       for y in range(by, min(by + block, H)) for x in range(bx, min(bx + block, W))}
            cnt = Counter(int(dl[j, i]) for i, j in parents)
            top = max(cnt.values())
            out[by:by + block, bx:bx + block] = 2 * min(v for v, n in cnt.items() if n == top)
    return out


@pytest.mark.parametrize("block", [2, 4, 8, 16])
def test_block_mode_counted(orc, block):
    rng = np.random.default_rng(block)
    for trial in range(6):
        Wc, Hc = int(rng.integers(3, 30)), int(rng.integers(3, 20))
        W, H = 2 * Wc + int(rng.integers(0, 2)), 2 * Hc + int(rng.integers(0, 2))
        dl = rng.integers(0, 6, size=(Hc, Wc)).astype(np.int16)  # few values: real modes and ties
        R, Dl = int(rng.choice([0, 4, 16])), 64
        lo, cap = orc.propagate_block(dl, W, H, Dl, R, block)
        ref = _block_mode_reference(dl, W, H, block)
        np.testing.assert_array_equal(lo, np.clip(ref - R, 0, Dl - cap))


def test_block_mode_hand_example(orc):
    # 4x4 coarse map, blocks of 4 fine pixels cover 2x2 parents
    dl = np.array([[3, 3, 1, 2],
                   [3, 7, 2, 1],
                   [5, 5, 9, 9],
                   [6, 6, 9, 0]], np.int16)
    lo, cap = orc.propagate_block(dl, 8, 8, 64, 0, 4)
    assert cap == 1
    # block modes: {3,3,3,7} -> 3; {1,2,2,1} -> tie 1/2 -> 1; {5,5,6,6} -> tie -> 5; {9,9,9,0} -> 9
    expect = np.kron(np.array([[6, 2], [10, 18]]), np.ones((4, 4), np.int64))
    np.testing.assert_array_equal(lo, expect)


def test_paper_propagation_wide_band_equals_single_scale(orc):
    """A radius that covers every level's range makes the paper's propagation, like any
    other, reduce to single-scale matching at the finest level."""
    from paper_2001_09678_amd.scene import make_scene
    sc = make_scene(8, 96, 64, 31, 5)
    ms = orc.pyramid(sc.left, sc.right, 32, levels=3, radius=64, num_paths=8, propagation="paper", block=8)[-1]
    ss = orc.pyramid(sc.left, sc.right, 32, levels=1, num_paths=8)[-1]
    np.testing.assert_array_equal(ms.out, ss.out)


def test_paper_propagation_schedule(orc):
    """The paper's d/4 scopes: every level below the top searches 2R+1 = D/4 + 1 disparities
    (radius D/8) around its propagated centre; the top searches D/4 (Section 3.4, eqs. Ot-O)."""
    from paper_2001_09678_amd.scene import make_scene
    sc = make_scene(9, 128, 96, 63, 6, ground=True)
    res = orc.pyramid(sc.left, sc.right, 64, levels=3, radius=8, num_paths=4, propagation="paper", block=8)
    assert [r.cap for r in res] == [16, 17, 17]
    assert [r.num_disp for r in res] == [16, 32, 64]
    # layer 1: blocks of 8 pixels share one band start; layer 2: interpolated per pixel
    lo1 = res[1].lo
    for by in range(0, lo1.shape[0], 8):
        for bx in range(0, lo1.shape[1], 8):
            assert len(np.unique(lo1[by:by + 8, bx:bx + 8])) == 1
    lo2, _ = orc.propagate_interp(res[1].dl, 128, 96, 64, 8)
    np.testing.assert_array_equal(res[2].lo, lo2)
