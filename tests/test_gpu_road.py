"""Road profile in v-disparity space (Section 3.5) on the HIP path vs the oracle, bit-exact,
through the C ABI: v- and u-disparity images of random and matched disparity maps (ragged
column tiles, pitched views, one disparity, the largest range), the road
Viterbi on random, line and ground-plane histograms, the degenerate cases (one disparity,
one row, eta = 2, eta beyond the height, unreachable ends), windows on both sides of the
narrow-window kernel (eta 9 and 10), heights at each change of rows per thread (1024,
2048) and the largest height."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2001_09678_amd import mpv as m, _lib
    _lib.lib()
    return m


@pytest.fixture(scope="module")
def road():
    from oracle import road as r
    return r


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("w,h,D", [(1, 1, 1), (37, 23, 16), (320, 240, 64), (1280, 720, 128), (100, 9, 256)])
def test_vdisparity(mpv, road, w, h, D):
    print("vdisparity", w, h, D, flush=True)
    rng = np.random.default_rng(w + h + D)
    disp = rng.integers(-1, D + 3, (h, w)).astype(np.int16)
    got = _np(mpv.vdisparity(_cuda(disp), D)).view(np.uint32)
    np.testing.assert_array_equal(got, road.vdisparity(disp, D))


def test_vdisparity_pitched_view(mpv, road):
    import torch
    rng = np.random.default_rng(3)
    full = rng.integers(-1, 40, (50, 90)).astype(np.int16)
    t = _cuda(full)[:, 7:71]  # a view with a row pitch larger than its width
    got = _np(mpv.vdisparity(t, 32)).view(np.uint32)
    np.testing.assert_array_equal(got, road.vdisparity(full[:, 7:71], 32))


@pytest.mark.parametrize("w,h,D", [(1, 1, 1), (37, 23, 16), (64, 5, 3), (65, 31, 64), (320, 240, 64),
                                   (1280, 720, 128), (100, 9, 256), (2000, 3, 256)])
def test_udisparity(mpv, road, w, h, D):
    print("udisparity", w, h, D, flush=True)
    rng = np.random.default_rng(7 * w + h + D)
    disp = rng.integers(-1, D + 3, (h, w)).astype(np.int16)
    got = _np(mpv.udisparity(_cuda(disp), D)).view(np.uint32)
    np.testing.assert_array_equal(got, road.udisparity(disp, D))


def test_udisparity_pitched_view(mpv, road):
    rng = np.random.default_rng(4)
    full = rng.integers(-1, 40, (50, 190)).astype(np.int16)
    t = _cuda(full)[:, 7:140]  # a view with a row pitch larger than its width
    got = _np(mpv.udisparity(t, 32)).view(np.uint32)
    np.testing.assert_array_equal(got, road.udisparity(full[:, 7:140], 32))


@pytest.mark.parametrize("D,H,eta", [(1, 1, 2), (1, 50, 3), (5, 1, 4), (6, 4, 3), (16, 40, 2), (48, 200, 6),
                                     (64, 200, 256), (128, 720, 8), (256, 4096, 3),
                                     # both sides of the narrow-window kernel (eta <= 9)
                                     (5, 12, 9), (40, 300, 9), (40, 300, 10), (3, 9, 10),
                                     # one, two and four rows per thread, both windows
                                     (20, 1024, 8), (20, 1025, 8), (64, 1080, 8), (32, 1500, 12),
                                     (16, 2048, 5), (16, 2049, 9), (12, 3000, 20)])
def test_road_random(mpv, road, D, H, eta):
    print("road", D, H, eta, flush=True)
    rng = np.random.default_rng(D * 7 + H + eta)
    hist = rng.integers(0, 5, (D, H)).astype(np.uint32)
    if D > 1 and H > 3 * D:  # a line to follow besides the noise
        hist[np.arange(D), 2 + 2 * np.arange(D)] += 9
    path, energy = mpv.road(_cuda(hist.view(np.int32)), eta)
    rp, re = road.road(hist, eta)
    np.testing.assert_array_equal(_np(path), rp)
    assert int(_np(energy)[0]) == re


def test_road_ties(mpv, road):
    """Flat histograms: every admissible path ties, so the smallest-row rules decide."""
    for D, H, eta in [(8, 30, 3), (20, 60, 4), (1, 10, 2)]:
        hist = np.ones((D, H), np.uint32)
        path, energy = mpv.road(_cuda(hist.view(np.int32)), eta)
        rp, re = road.road(hist, eta)
        np.testing.assert_array_equal(_np(path), rp)
        assert int(_np(energy)[0]) == re


def test_road_of_a_matched_scene(mpv, road):
    """The 1280x720, D=128 workload: its LR-checked map, its v- and u-disparity images and
    its road profile, each against the oracle applied to the previous GPU output."""
    from paper_2001_09678_amd.scene import config_scene
    sc, cfg = config_scene("c2")
    p = mpv.MPVParams(num_disp=128, num_paths=8)
    disp = mpv.pyramid(_cuda(sc.left), _cuda(sc.right), p, levels=3, radius=4).disp
    hist = mpv.vdisparity(disp, 128)
    np.testing.assert_array_equal(_np(hist).view(np.uint32), road.vdisparity(_np(disp), 128))
    uh = mpv.udisparity(disp, 128)
    np.testing.assert_array_equal(_np(uh).view(np.uint32), road.udisparity(_np(disp), 128))
    path, energy = mpv.road(hist, 8)
    rp, re = road.road(_np(hist).view(np.uint32), 8)
    np.testing.assert_array_equal(_np(path), rp)
    assert int(_np(energy)[0]) == re
