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


@pytest.mark.parametrize("tight", [False, True])
def test_service_results_equal_solo(rigs, tight):
    from paper_2001_09678_amd import serve
    specs, frames, solo = rigs
    _log("serve tight" if tight else "serve roomy", [(s.width, s.height, s.num_disp) for s in specs])
    ex = serve.GpuExecutor(streams=2)
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
