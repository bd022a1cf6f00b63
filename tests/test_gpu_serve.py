"""Frame-stream service on the GPU: every frame's result is bit-identical to the same frame
matched alone, under a roomy and a tight HBM budget; an injected fault fails only its request;
the solo result of one frame of every rig equals the oracle, so the service's results do too."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def rigs():
    import torch
    assert torch.cuda.is_available()
    from paper_2001_09678_amd import serve, mpv
    specs = serve.rig_specs(8, 5)
    frames = serve.rig_frames(specs, 2, pinned=True)
    solo = []
    for sp, fr in zip(specs, frames):
        params = mpv.MPVParams(num_disp=sp.num_disp, num_paths=8)
        outs = []
        for l, r in fr:
            p = mpv.pyramid(l.cuda(), r.cuda(), params, levels=3, radius=4)
            outs.append(p.disp.cpu().numpy())
        solo.append(outs)
    return specs, frames, solo


def test_rig_frames_equal_oracle(rigs, orc):
    """Frame 0 of each of the 8 rigs (640x360 .. 1920x1080, D 64 .. 256) matched on the GPU
    equals the oracle bit for bit."""
    specs, frames, solo = rigs
    for i, (sp, fr) in enumerate(zip(specs, frames)):
        _log("oracle for rig", i, (sp.width, sp.height, sp.num_disp))
        l, r = fr[0]
        ref = orc.pyramid(l.numpy(), r.numpy(), sp.num_disp, levels=3, radius=4, num_paths=8)[-1]
        np.testing.assert_array_equal(solo[i][0], ref.out, err_msg=f"rig {i} vs oracle")


def _make(specs, frames, inject=()):
    from paper_2001_09678_amd import serve

    def make(rid, rig, seq, t):
        l, r = frames[rig][seq % len(frames[rig])]
        return serve.Request(rid, rig, seq, specs[rig], l, r, t,
                             inject="launch" if (rig, seq) in inject else None)
    return make


@pytest.mark.parametrize("kind", ["streams", "batched"])
@pytest.mark.parametrize("tight", [False, True])
def test_service_results_equal_solo(rigs, tight, kind):
    from paper_2001_09678_amd import serve
    specs, frames, solo = rigs
    _log("serve", kind, "tight" if tight else "roomy", [(s.width, s.height, s.num_disp) for s in specs])
    ex = serve.GpuExecutor(streams=2) if kind == "streams" else serve.BatchedGpuExecutor(specs, per_spec=3)
    need = sorted(ex.bytes_needed(s) for s in specs)
    budget = need[-1] + need[-2] if tight else 8 << 30
    server = serve.Server(ex, budget, max_inflight=16, max_batch=8)
    sched = serve.arrivals(8, 30.0, 0.5, seed=5)
    res = serve.run(server, sched, _make(specs, frames, inject={(0, 3)}))
    assert len(res) == len(sched)
    assert server.pool.peak <= budget
    for r in res:
        if (r.rig, r.seq) == (0, 3):
            assert not r.ok and "injected" in r.error
            continue
        assert r.ok, r.error
        np.testing.assert_array_equal(r.disp, solo[r.rig][r.seq % 2])
    s = serve.latency_summary(res, 0.5)
    _log("latency", s, "launches", server.launches, "peak bytes", server.pool.peak)
    server.close()
    if kind == "batched":
        assert ex.launches["lone"] > 0  # light load: the lane-group batch serves lone frames
        ex.close()


def test_batched_service_saturated_equals_solo(rigs):
    """Every frame offered at once: admission steps carry several frames of mixed shapes into
    one batched launch, and every result still equals the frame matched alone."""
    from paper_2001_09678_amd import serve
    specs, frames, solo = rigs
    ex = serve.BatchedGpuExecutor(specs, per_spec=4)
    server = serve.Server(ex, 16 << 30, max_inflight=32, max_batch=16)
    sched = [(0.0, r, f) for f in range(4) for r in range(8)]
    res = serve.run(server, sched, _make(specs, frames))
    assert len(res) == len(sched) and all(r.ok for r in res)
    for r in res:
        np.testing.assert_array_equal(r.disp, solo[r.rig][r.seq % 2])
    assert max(server.batch_sizes) > 1
    assert ex.launches["batched"] > 0  # steps of several frames take the batched layouts
    _log("batched saturated: launches", server.launches, "mean batch",
         sum(server.batch_sizes) / len(server.batch_sizes), ex.launches)
    server.close()
    ex.close()


def test_invalid_request_fails_alone(rigs):
    from paper_2001_09678_amd import serve
    specs, frames, solo = rigs
    ex = serve.GpuExecutor(streams=1)
    server = serve.Server(ex, 8 << 30)
    bad = serve.FrameSpec(specs[0].width, specs[0].height, 1000)
    specs2 = [specs[0], bad]
    frames2 = [frames[0], frames[0]]
    sched = [(0.0, 0, 0), (0.0, 1, 0), (0.001, 0, 1)]
    res = {(r.rig, r.seq): r for r in serve.run(server, sched, _make(specs2, frames2))}
    assert not res[(1, 0)].ok and "invalid" in res[(1, 0)].error
    np.testing.assert_array_equal(res[(0, 0)].disp, solo[0][0])
    np.testing.assert_array_equal(res[(0, 1)].disp, solo[0][1])
    server.close()


def test_learned_service_equals_solo(rigs):
    """The learned-band path with plain fallback in the service (proposal, then the banded
    finest level or full range once the proposal's count reaches the host, no blocking read):
    every frame equals the learned matcher run on that frame alone, and the fallback fraction
    is reported."""
    import torch
    from paper_2001_09678_amd import learned, mpv, serve
    specs, frames, _ = rigs
    net, _ = learned.BandNet.load(learned.DEFAULT_WEIGHTS)
    solo = []
    for sp, fr in zip(specs, frames):
        m = learned.LearnedMatcher(net, mpv.MPVParams(num_disp=sp.num_disp, num_paths=8), sp.width, sp.height)
        solo.append([m(l.cuda(), r.cuda()).cpu().numpy() for l, r in fr])
    ex = serve.LearnedGpuExecutor(net, streams=2)
    server = serve.Server(ex, 16 << 30, max_inflight=8, max_batch=4)
    sched = serve.arrivals(8, 30.0, 0.3, seed=5)
    res = serve.run(server, sched, _make(specs, frames))
    assert len(res) == len(sched)
    for r in res:
        assert r.ok, r.error
        np.testing.assert_array_equal(r.disp, solo[r.rig][r.seq % 2], err_msg=f"rig {r.rig} frame {r.seq}")
    assert ex.frames == len(res) and 0.0 <= ex.fallback_fraction <= 1.0
    _log("learned service: fallback fraction", ex.fallback_fraction)
    server.close()
