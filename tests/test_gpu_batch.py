"""Batched multi-pair execution and launch schedules, through the C ABI.

* every pair of a batch (mixed sizes and ranges) equals its solo mpv_pyramid result and the
  oracle, bit for bit, for every schedule;
* graph replays: the captured batch replayed several times, with eager work and
  synchronisations in between, matches the eager run each time;
* schedule invariance: every schedule an autotuner may pick gives identical bits;
* the 64-pair workload (640x360 / 1280x720 / 1920x1080, D in {64, 128, 256}) at full size:
  every pair equals its solo run, and one pair of each of the 9 (size, range) combinations
  equals the oracle.
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


SMALL = [(96, 64, 32), (131, 75, 48), (200, 117, 128), (64, 40, 64), (150, 90, 96), (131, 75, 40)]
SCHEDULES = [dict(), dict(waves_per_block=4, order=1), dict(waves_per_block=2, order=0),
             dict(full_lanes=32, band_lanes=32, order=1)]


def _small_scenes():
    from paper_2001_09678_amd.scene import make_scene
    return [make_scene(70 + i, w, h, d - 1, 6, ground=True) for i, (w, h, d) in enumerate(SMALL)]


@pytest.mark.parametrize("sched", range(len(SCHEDULES)))
def test_batch_equals_solo_and_oracle(mpv, orc, sched):
    _log("batch small, schedule", SCHEDULES[sched])
    scenes = _small_scenes()
    params = mpv.MPVParams(num_disp=64, num_paths=8)
    s = mpv.Schedule(**SCHEDULES[sched])
    pairs = [(_cuda(sc.left), _cuda(sc.right), d) for sc, (_, _, d) in zip(scenes, SMALL)]
    b = mpv.Batch(pairs, params, levels=3, radius=4, sched=s, want_all=True)
    b.run()
    for i, (sc, (w, h, d)) in enumerate(zip(scenes, SMALL)):
        got = _np(b.disp[i])
        solo = mpv.pyramid(pairs[i][0], pairs[i][1], mpv.MPVParams(num_disp=d, num_paths=8), levels=3,
                           radius=4)
        np.testing.assert_array_equal(got, _np(solo.disp), err_msg=f"pair {i} vs solo")
        ref = orc.pyramid(sc.left, sc.right, d, levels=3, radius=4, num_paths=8)[-1]
        np.testing.assert_array_equal(got, ref.out, err_msg=f"pair {i} vs oracle")
        np.testing.assert_array_equal(_np(b.raw[i]), ref.dl)
        np.testing.assert_array_equal(_np(b.right[i]), ref.dr)


def test_batch_graph_replays(mpv):
    """Capture once, replay with new inputs written between replays (eager work), each
    replay checked against an eager run on the same inputs."""
    import torch
    from paper_2001_09678_amd.scene import make_scene
    _log("batch graph replays")
    params = mpv.MPVParams(num_disp=64, num_paths=8)
    lefts = [torch.empty((h, w), dtype=torch.uint8, device="cuda") for (w, h, _) in SMALL]
    rights = [torch.empty_like(t) for t in lefts]
    pairs = [(l, r, d) for l, r, (_, _, d) in zip(lefts, rights, SMALL)]
    gb = mpv.Batch(pairs, params, levels=3, radius=4, sched=mpv.Schedule(order=1))
    eb = mpv.Batch(pairs, params, levels=3, radius=4)
    for rep in range(3):
        for i, (w, h, d) in enumerate(SMALL):
            sc = make_scene(500 + 10 * rep + i, w, h, d - 1, 5, ground=rep % 2 == 0)
            lefts[i].copy_(_cuda(sc.left))
            rights[i].copy_(_cuda(sc.right))
        torch.cuda.synchronize()
        gb.run_graph()
        torch.cuda.synchronize()
        eb.run()
        torch.cuda.synchronize()
        for i in range(len(SMALL)):
            np.testing.assert_array_equal(_np(gb.disp[i]), _np(eb.disp[i]), err_msg=f"replay {rep} pair {i}")
        assert any((_np(t) >= 0).any() for t in gb.disp)


@pytest.mark.parametrize("levels,sched", [
    (3, dict(waves_per_block=4)), (3, dict(waves_per_block=2, band_lanes=32)), (3, dict(band_lanes=64)),
    (1, dict(full_lanes=32)), (1, dict(full_lanes=32, waves_per_block=4)),
])
def test_schedule_invariance_full_size(mpv, levels, sched):
    """1280x720, D=128, 8 paths: every schedule gives the default schedule's bits."""
    from paper_2001_09678_amd.scene import config_scene
    _log("schedule invariance", levels, sched)
    sc, cfg = config_scene("c2")
    L, R = _cuda(sc.left), _cuda(sc.right)
    params = mpv.MPVParams(num_disp=128, num_paths=8)
    ref = mpv.pyramid(L, R, params, levels=levels, radius=4)
    got = mpv.pyramid(L, R, params, levels=levels, radius=4, sched=mpv.Schedule(**sched))
    np.testing.assert_array_equal(_np(got.disp), _np(ref.disp))
    np.testing.assert_array_equal(_np(got.right), _np(ref.right))
    np.testing.assert_array_equal(_np(got.raw), _np(ref.raw))


@pytest.fixture(scope="module")
def batch_workload(mpv):
    """The 64-pair workload at its full sizes in the launch configuration the benchmark
    times (graph replay, longest lines first); returns specs, scenes and every pair's map."""
    from paper_2001_09678_amd.scene import batch_specs, batch_scenes
    specs = batch_specs()
    _log("batch workload: generating", len(specs), "scenes")
    scenes = batch_scenes(specs, workers=16)
    params = mpv.MPVParams(num_disp=128, num_paths=8)
    pairs = [(_cuda(sc.left), _cuda(sc.right), sp[3]) for sc, sp in zip(scenes, specs)]
    _log("batch workload: run")
    b = mpv.Batch(pairs, params, levels=3, radius=4, sched=mpv.Schedule(waves_per_block=4, order=1))
    b.run_graph()
    got = [_np(t) for t in b.disp]
    return specs, scenes, pairs, got


def test_batch_workload_full_size(mpv, batch_workload):
    """Every pair of the 64-pair batch equals its solo run."""
    specs, scenes, pairs, got = batch_workload
    for i, sp in enumerate(specs):
        solo = mpv.pyramid(pairs[i][0], pairs[i][1], mpv.MPVParams(num_disp=sp[3], num_paths=8),
                           levels=3, radius=4)
        np.testing.assert_array_equal(got[i], _np(solo.disp), err_msg=f"pair {i} {sp}")


BATCH_COMBOS = [(w, h, d) for (w, h) in [(640, 360), (1280, 720), (1920, 1080)] for d in (64, 128, 256)]


@pytest.mark.parametrize("combo", BATCH_COMBOS, ids=[f"{w}x{h}_D{d}" for w, h, d in BATCH_COMBOS])
def test_batch_workload_vs_oracle(orc, batch_workload, combo):
    """The first pair of each (size, range) combination of the 64-pair batch equals the
    oracle bit for bit (the batch's descriptors, per-pair ranges and workspace regions)."""
    specs, scenes, _, got = batch_workload
    idx = [i for i, sp in enumerate(specs) if (sp[1], sp[2], sp[3]) == combo]
    assert idx, f"the workload draws no pair of {combo}"
    i = idx[0]
    _log("oracle for pair", i, specs[i])
    ref = orc.pyramid(scenes[i].left, scenes[i].right, specs[i][3], levels=3, radius=4, num_paths=8)[-1]
    np.testing.assert_array_equal(got[i], ref.out, err_msg=f"pair {i} {specs[i]} vs oracle")


def test_run_items_subsets(mpv, orc):
    """mpv_batch_run_items: successive runs over different subsets (in any order, more than
    the staging ring holds) each give the solo results of exactly their pairs and leave the
    other pairs' outputs untouched; a full run afterwards still works."""
    import torch
    scenes = _small_scenes()
    params = mpv.MPVParams(num_disp=64, num_paths=8)
    pairs = [(_cuda(sc.left), _cuda(sc.right), d) for sc, (_, _, d) in zip(scenes, SMALL)]
    solo = [_np(mpv.pyramid(l, r, mpv.MPVParams(num_disp=d, num_paths=8), levels=3, radius=4).disp)
            for l, r, d in pairs]
    b = mpv.Batch(pairs, params, levels=3, radius=4, sched=mpv.Schedule(waves_per_block=2, order=1))
    subsets = [[3], [0, 5], [4, 1, 2], [5], [2, 0], [1, 3, 4, 5], [0]]
    for sub in subsets:
        _log("run_items", sub)
        for t in b.disp:
            t.fill_(-9)
        b.run_items(sub)
        torch.cuda.synchronize()
        for i in range(len(pairs)):
            got = _np(b.disp[i])
            if i in sub:
                np.testing.assert_array_equal(got, solo[i], err_msg=f"subset {sub} pair {i}")
            else:
                assert (got == -9).all(), f"subset {sub} touched pair {i}"
    b.run()
    for i in range(len(pairs)):
        np.testing.assert_array_equal(_np(b.disp[i]), solo[i])
    ref = orc.pyramid(scenes[2].left, scenes[2].right, SMALL[2][2], levels=3, radius=4, num_paths=8)[-1]
    np.testing.assert_array_equal(_np(b.disp[2]), ref.out)
