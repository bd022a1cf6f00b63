"""Frame-stream service on the CPU: a simulated executor (oracle results, modelled service
times) on a virtual clock. Admission never exceeds the budget, FIFO order holds, frames join
while others are in flight, faults fail only their own request, latencies are bookkept."""
import numpy as np
import pytest

import oracle
from paper_2001_09678_amd import serve
from paper_2001_09678_amd.scene import make_scene


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Service time a + b*W*H*D per frame, frames of one launch run back to back on one of
    `streams` simulated streams; results come from the oracle (small frames only)."""

    def __init__(self, clock, streams=2, a=50e-6, b=1e-9, compute=False):
        self.clock, self.a, self.b, self.compute = clock, a, b, compute
        self.free_at = [0.0] * streams
        self.k = 0
        self.allocs = self.frees = 0
        self.live = {}

    def bytes_needed(self, spec):
        if spec.num_disp > 256 or spec.width < 8 or spec.height < 8:
            return 0
        return spec.width * spec.height * (2 + spec.num_disp // 8)

    def alloc(self, spec):
        self.allocs += 1
        slot = {"spec": spec, "id": self.allocs}
        self.live[slot["id"]] = slot
        return slot

    def free(self, slot):
        self.frees += 1
        del self.live[slot["id"]]

    def launch(self, items):
        s = self.k % len(self.free_at)
        self.k += 1
        t = max(self.clock(), self.free_at[s])
        out = []
        for req, slot in items:
            if req.inject == "launch":
                out.append(RuntimeError("injected launch fault"))
                continue
            sp = req.spec
            t += self.a + self.b * sp.width * sp.height * sp.num_disp
            out.append((t, req))
        self.free_at[s] = t
        return out

    def done(self, ticket):
        return isinstance(ticket, Exception) or self.clock() >= ticket[0] - 1e-12

    def collect(self, ticket):
        if isinstance(ticket, Exception):
            return ticket
        req = ticket[1]
        if not self.compute:
            return None
        r = oracle.pyramid(req.left, req.right, req.spec.num_disp, levels=2, num_paths=4)
        return r[-1].out

    def next_done(self, inflight):
        ts = [tk[0] for tk, *_ in inflight if not isinstance(tk, Exception)]
        return min(ts) if ts else None


def _drive(server, ex, clock, schedule, make_request, deadline_s=None):
    def wait(nxt):
        cands = [x for x in (nxt, ex.next_done(server.inflight)) if x is not None]
        if cands:
            clock.t = max(clock.t, min(cands))
        else:
            clock.t += 1e-4
    return serve.run(server, schedule, make_request, clock=clock, wait=wait, deadline_s=deadline_s)


def _requests(specs, images=None, inject=None):
    def make(rid, rig, seq, t):
        sp = specs[rig]
        l, r = images[rig] if images else (None, None)
        return serve.Request(rid, rig, seq, sp, l, r, t, inject=(inject or {}).get((rig, seq)))
    return make


def test_arrivals_and_rig_specs():
    sched = serve.arrivals(8, 30.0, 2.0, seed=5)
    assert sched == sorted(sched)
    per = np.bincount([r for _, r, _ in sched], minlength=8)
    assert (per >= 59).all() and (per <= 61).all()
    for r in range(8):
        ts = np.array([t for t, rr, _ in sched if rr == r])
        gaps = np.diff(ts)
        assert (np.abs(gaps - 1 / 30) <= 2e-3 + 1e-12).all()
    specs = serve.rig_specs(8, 5)
    assert specs == serve.rig_specs(8, 5)
    assert all((s.width, s.height) in serve.RESOLUTIONS and s.num_disp in serve.RANGES for s in specs)


def test_budget_never_exceeded_and_fifo():
    clock = Clock()
    ex = FakeExecutor(clock)
    specs = serve.rig_specs(8, 5)
    need = [ex.bytes_needed(s) for s in specs]
    budget = 2 * max(need) + min(need)   # tight: a few frames in flight at most
    server = serve.Server(ex, budget, max_inflight=16, max_batch=4, clock=clock)
    pool = server.pool
    orig = pool.acquire

    def checked(spec):
        got = orig(spec)
        assert pool.held <= budget and pool.busy <= pool.held
        return got
    pool.acquire = checked
    res = _drive(server, ex, clock, serve.arrivals(8, 30.0, 1.0, seed=5), _requests(specs))
    assert len(res) == len(serve.arrivals(8, 30.0, 1.0, seed=5))
    assert all(r.ok for r in res)
    assert pool.peak <= budget
    # admission is FIFO: admit times never decrease with request id
    adm = [r.t_admit for r in sorted(res, key=lambda r: r.rid)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))
    # device memory is bounded by the budget: live slots never exceed it
    assert sum(ex.bytes_needed(s["spec"]) for s in ex.live.values()) <= budget
    server.close()
    assert not ex.live


def test_latency_bookkeeping_without_contention():
    clock = Clock()
    ex = FakeExecutor(clock, a=1e-3, b=0.0)
    spec = serve.FrameSpec(64, 48, 16)
    server = serve.Server(ex, 1 << 30, clock=clock)
    sched = [(0.01 * i, 0, i) for i in range(20)]
    res = _drive(server, ex, clock, sched, _requests([spec]))
    lat = sorted(r.latency for r in res)
    assert all(abs(x - 1e-3) < 1e-9 for x in lat)
    s = serve.latency_summary(res, 0.2)
    assert s["ok"] == 20 and abs(s["p50_ms"] - 1.0) < 1e-6 and abs(s["p99_ms"] - 1.0) < 1e-6


def test_continuous_batching_joins_while_others_run():
    clock = Clock()
    ex = FakeExecutor(clock, streams=2, a=10e-3, b=0.0)
    spec = serve.FrameSpec(64, 48, 16)
    server = serve.Server(ex, 1 << 30, max_inflight=8, max_batch=8, clock=clock)
    sched = [(0.0, 0, 0), (0.0, 1, 0), (0.002, 2, 0)]
    res = {r.rig: r for r in _drive(server, ex, clock, sched, _requests([spec] * 3))}
    # the late frame is admitted at its arrival, before the first batch completes
    assert res[2].t_admit < res[0].t_done
    assert res[2].t_admit == pytest.approx(0.002)
    # and runs on the other stream: it does not wait for the first launch
    assert res[2].t_done == pytest.approx(0.012)


def test_faults_fail_only_their_requests():
    clock = Clock()
    ex = FakeExecutor(clock)
    good = serve.FrameSpec(64, 48, 16)
    bad_range = serve.FrameSpec(64, 48, 1000)
    huge = serve.FrameSpec(4096, 4096, 256)
    specs = [good, bad_range, huge, good]
    budget = 10 * ex.bytes_needed(good)
    server = serve.Server(ex, budget, clock=clock)
    sched = [(0.001 * i, i % 4, i // 4) for i in range(40)]
    res = _drive(server, ex, clock, sched, _requests(specs, inject={(3, 2): "launch", (0, 5): "launch"}))
    by = {(r.rig, r.seq): r for r in res}
    assert len(by) == 40
    for (rig, seq), r in by.items():
        if rig == 1:
            assert not r.ok and "invalid" in r.error
        elif rig == 2:
            assert not r.ok and "budget" in r.error
        elif (rig, seq) in ((3, 2), (0, 5)):
            assert not r.ok and "injected" in r.error
        else:
            assert r.ok, (rig, seq, r.error)


def test_deadline_expires_in_queue_only():
    clock = Clock()
    ex = FakeExecutor(clock, streams=1, a=5e-3, b=0.0)
    spec = serve.FrameSpec(64, 48, 16)
    server = serve.Server(ex, 1 << 30, max_inflight=1, max_batch=1, clock=clock)
    sched = [(0.0, 0, i) for i in range(6)]   # a burst; one in flight at a time
    res = _drive(server, ex, clock, sched, _requests([spec]), deadline_s=0.012)
    ok = sorted(r.seq for r in res if r.ok)
    expired = sorted(r.seq for r in res if not r.ok)
    assert ok == [0, 1, 2] and expired == [3, 4, 5]
    assert all("expired" in r.error for r in res if not r.ok)


def test_results_equal_solo_oracle():
    """The simulated executor returns oracle results; each frame's result in the mix equals
    the same frame matched alone."""
    clock = Clock()
    ex = FakeExecutor(clock, compute=True)
    specs = [serve.FrameSpec(48, 32, 16), serve.FrameSpec(40, 24, 16)]
    images = []
    for i, sp in enumerate(specs):
        sc = make_scene(900 + i, sp.width, sp.height, sp.num_disp - 1, 4)
        images.append((sc.left, sc.right))
    server = serve.Server(ex, 1 << 30, clock=clock)
    sched = serve.arrivals(2, 30.0, 0.2, seed=1)
    res = _drive(server, ex, clock, sched, _requests(specs, images))
    for r in res:
        sp = specs[r.rig]
        solo = oracle.pyramid(images[r.rig][0], images[r.rig][1], sp.num_disp, levels=2, num_paths=4)[-1].out
        np.testing.assert_array_equal(r.disp, solo)
