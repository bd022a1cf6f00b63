"""One scan line per lane in batches (mpv_schedule.band_lanes = MPV_BAND_LANES_LINE), through
the C ABI.

A batched banded level's vertical and diagonal directions run with one line per lane, 64
neighbouring lines per wave walked row by row, while the horizontal directions' 16-lane groups
run beside them on a second stream. A pixel's partials are six-bit slots in 8 bytes where
every normalised energy fits (24 + lambda*tau <= 63), else 12 byte slots. Against the oracle
bit for bit (the finest level's raw winners, right disparities and LR-checked map): both band
lengths with kernels (5 and 9), the three compile-time reduced taus, both slot layouts (and
the largest energy six bits hold), 4 and 8 paths, ragged
waves at the end of a direction, lines that start and end on different rows, tall and narrow
images (every diagonal line starts on a side), rows shorter than the disparity range; at full
size against the default layout for one pair, the 16-frame batch (eager and graph replay) and
a mixed batch. Levels the layout does not take (other band lengths or taus, layered merges,
gradient weights) and single-pair entry points must run as with the default schedule.
"""
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


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _log(*a):
    print(*a, flush=True)


def _line(mpv, **kw):
    return mpv.Schedule(band_lanes=mpv.Schedule.LINE, **kw)


def _batch1(mpv, L, R, D, params, levels, radius, sched):
    b = mpv.Batch([(L, R, D)], params, levels=levels, radius=radius, sched=sched, want_all=True)
    b.run()
    return b


# (width, height, D, levels, radius, paths, tau, lambda)
CASES = [
    (160, 96, 64, 3, 4, 8, 4, 8),
    (131, 75, 48, 3, 4, 8, 4, 8),
    (61, 150, 32, 2, 4, 8, 4, 8),
    (200, 40, 64, 3, 2, 8, 4, 8),
    (97, 61, 64, 3, 4, 4, 4, 8),
    (150, 90, 96, 3, 4, 8, 2, 10),
    (150, 90, 96, 3, 2, 8, 1, 20),
    (70, 9, 40, 2, 4, 8, 4, 8),
    (5, 33, 16, 2, 2, 8, 4, 8),
    (129, 65, 128, 2, 4, 8, 4, 8),
    (163, 99, 64, 3, 4, 8, 4, 8),
    (300, 70, 256, 3, 4, 8, 4, 7),
    # 24 + lambda*tau = 63: the largest energy the six-bit slots hold; 64 and 72: 12-byte slots
    (131, 75, 48, 3, 4, 8, 1, 39),
    (131, 75, 48, 3, 4, 8, 1, 40),
    (150, 90, 96, 3, 4, 8, 4, 12),
    (97, 61, 64, 3, 4, 4, 2, 20),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}_D{c[2]}_L{c[3]}_R{c[4]}_P{c[5]}_t{c[6]}" for c in CASES])
def test_line_layout_vs_oracle(mpv, orc, case):
    """A one-pair batch with one line per lane against the oracle: raw winners, right
    disparities and the LR-checked map of the finest level."""
    from paper_2001_09678_amd.scene import make_scene
    w, h, D, levels, R, P, tau, lam = case
    _log("line layout", case)
    sc = make_scene(900 + w + h, w, h, D - 1, 6, ground=True)
    p = mpv.MPVParams(num_disp=D, num_paths=P, lam=lam, tau=tau)
    b = _batch1(mpv, _cuda(sc.left), _cuda(sc.right), D, p, levels, R, _line(mpv, waves_per_block=2))
    ref = orc.pyramid(sc.left, sc.right, D, levels=levels, radius=R, num_paths=P, lam=lam, tau=tau)[-1]
    np.testing.assert_array_equal(_np(b.raw[0]), ref.dl)
    np.testing.assert_array_equal(_np(b.right[0]), ref.dr)
    np.testing.assert_array_equal(_np(b.disp[0]), ref.out)


@pytest.mark.parametrize("wpb", [1, 2, 4])
def test_line_layout_full_size(mpv, wpb):
    """1280x720, D=128, 3 levels, +/-4 bands, one pair: identical to the default layout."""
    from paper_2001_09678_amd.scene import config_scene
    _log("line layout full size, waves per block", wpb)
    sc, _ = config_scene("c2")
    L, R = _cuda(sc.left), _cuda(sc.right)
    params = mpv.MPVParams(num_disp=128, num_paths=8)
    ref = _batch1(mpv, L, R, 128, params, 3, 4, mpv.Schedule(waves_per_block=wpb))
    got = _batch1(mpv, L, R, 128, params, 3, 4, _line(mpv, waves_per_block=wpb))
    np.testing.assert_array_equal(_np(got.raw[0]), _np(ref.raw[0]))
    np.testing.assert_array_equal(_np(got.right[0]), _np(ref.right[0]))
    np.testing.assert_array_equal(_np(got.disp[0]), _np(ref.disp[0]))


def test_line_layout_workload_oracle(mpv, orc):
    """The 1280x720, D=128 workload's pair against the oracle with one line per lane."""
    from paper_2001_09678_amd.scene import config_scene
    sc, _ = config_scene("c2")
    _log("line layout vs oracle, 1280x720")
    b = _batch1(mpv, _cuda(sc.left), _cuda(sc.right), 128, mpv.MPVParams(num_disp=128, num_paths=8), 3, 4,
                _line(mpv, waves_per_block=4))
    ref = orc.pyramid(sc.left, sc.right, 128, levels=3, radius=4, num_paths=8)[-1]
    np.testing.assert_array_equal(_np(b.raw[0]), ref.dl)
    np.testing.assert_array_equal(_np(b.disp[0]), ref.out)


def test_line_layout_step_batch(mpv):
    """The benchmark's 16-frame batch (eager and graph replay): every frame identical to the
    default layout's batch."""
    from paper_2001_09678_amd.scene import config_specs, config_scene
    import torch
    specs = config_specs("c2", 16)
    _log("16-frame batch, line layout")
    pairs = []
    for sp in specs:
        sc, _ = config_scene("c2", sp[0])
        pairs.append((_cuda(sc.left), _cuda(sc.right), sp[3]))
    params = mpv.MPVParams(num_disp=128, num_paths=8)
    ref = mpv.Batch(pairs, params, levels=3, radius=4, sched=mpv.Schedule(waves_per_block=4, order=1))
    ref.run()
    want = [_np(t) for t in ref.disp]
    got = mpv.Batch(pairs, params, levels=3, radius=4, sched=_line(mpv, waves_per_block=4, order=1))
    got.run()
    for i in range(len(pairs)):
        np.testing.assert_array_equal(_np(got.disp[i]), want[i], err_msg=f"frame {i}")
    for t in got.disp:
        t.fill_(-9)
    torch.cuda.synchronize()
    got.run_graph()
    got.run_graph()
    for i in range(len(pairs)):
        np.testing.assert_array_equal(_np(got.disp[i]), want[i], err_msg=f"graph frame {i}")


def test_line_layout_mixed_batch(mpv, orc):
    """Pairs of mixed sizes and ranges in one batch: solo results and the oracle."""
    from paper_2001_09678_amd.scene import make_scene
    small = [(96, 64, 32), (131, 75, 48), (200, 117, 128), (64, 40, 64), (150, 90, 96), (33, 70, 40)]
    scenes = [make_scene(70 + i, w, h, d - 1, 6, ground=True) for i, (w, h, d) in enumerate(small)]
    pairs = [(_cuda(sc.left), _cuda(sc.right), d) for sc, (_, _, d) in zip(scenes, small)]
    b = mpv.Batch(pairs, mpv.MPVParams(num_disp=64, num_paths=8), levels=3, radius=4,
                  sched=_line(mpv, waves_per_block=2, order=1), want_all=True)
    b.run()
    for i, (sc, (w, h, d)) in enumerate(zip(scenes, small)):
        _log("mixed batch pair", i, (w, h, d))
        ref = orc.pyramid(sc.left, sc.right, d, levels=3, radius=4, num_paths=8)[-1]
        np.testing.assert_array_equal(_np(b.disp[i]), ref.out, err_msg=f"pair {i}")
        np.testing.assert_array_equal(_np(b.raw[i]), ref.dl, err_msg=f"pair {i} raw")
        np.testing.assert_array_equal(_np(b.right[i]), ref.dr, err_msg=f"pair {i} right")


@pytest.mark.parametrize("kw", [dict(merge="layered"), dict(grad_sigma=16), dict(radius=3), dict(tau=3)],
                         ids=["layered", "grad", "cap7", "tau3"])
def test_line_schedule_elsewhere_unchanged(mpv, kw):
    """Where the layout does not apply, a batch with the schedule gives the default's bits,
    and so does a single pair through mpv_pyramid (which never takes it)."""
    from paper_2001_09678_amd.scene import make_scene
    kw = dict(kw)
    radius = kw.pop("radius", 4)
    sc = make_scene(44, 150, 90, 63, 6, ground=True)
    L, R = _cuda(sc.left), _cuda(sc.right)
    p = mpv.MPVParams(num_disp=64, num_paths=8, **kw)
    _log("line schedule elsewhere", kw, radius)
    ref = _batch1(mpv, L, R, 64, p, 3, radius, mpv.Schedule())
    got = _batch1(mpv, L, R, 64, p, 3, radius, _line(mpv))
    np.testing.assert_array_equal(_np(got.disp[0]), _np(ref.disp[0]))
    np.testing.assert_array_equal(_np(got.raw[0]), _np(ref.raw[0]))
    solo = mpv.pyramid(L, R, p, levels=3, radius=radius, sched=_line(mpv))
    np.testing.assert_array_equal(_np(solo.disp), _np(ref.disp[0]))


def test_line_schedule_single_pair_is_default(mpv):
    """mpv_pyramid with the schedule runs the default layout (a lone frame's lines would be
    long serial chains): identical bits, SSIM data term included."""
    from paper_2001_09678_amd.scene import make_scene
    sc = make_scene(45, 150, 90, 63, 6, ground=True)
    L, R = _cuda(sc.left), _cuda(sc.right)
    for p in (mpv.MPVParams(num_disp=64, num_paths=8), mpv.MPVParams(num_disp=64, num_paths=8, data_term="ssim")):
        ref = mpv.pyramid(L, R, p, levels=3, radius=4)
        got = mpv.pyramid(L, R, p, levels=3, radius=4, sched=_line(mpv))
        np.testing.assert_array_equal(_np(got.disp), _np(ref.disp))
