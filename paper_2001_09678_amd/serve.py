"""Frame-stream service: several camera rigs, HBM-budget admission, continuous batching.

The counterpart of the paper's real-time pipeline (Section 3.7: frames captured and matched
while the previous ones are still in flight), for many rigs sharing one GPU:

* rigs deliver frames at a fixed rate (random phase, small jitter);
* a FIFO admission queue admits the head frame while a slot for its shape fits in the HBM
  budget (inputs, pyramid workspace and outputs of one in-flight frame; idle slots of other
  shapes are evicted first) and fewer than `max_inflight` frames are in flight;
* admitted frames are launched at once, round-robin over k streams: upload, multi-scale MPV,
  download, each frame completing on its own event. A frame joins whenever a slot frees;
  no frame waits for a whole batch to finish (continuous batching);
* a request fails alone: an invalid shape or range, a request larger than the whole budget,
  an error raised while launching it, or a deadline passed in the queue.

Latency is arrival to the host seeing its download complete. The scheduler is written
against an executor interface (bytes_needed / alloc / free / launch / done / collect) and a
clock, so admission, batching, fault handling and latency bookkeeping also run on the CPU
with a simulated executor and a virtual clock.
"""
from __future__ import annotations

import time
from collections import OrderedDict, deque
from dataclasses import dataclass, field

import numpy as np

__all__ = ["FrameSpec", "Request", "Result", "SlotPool", "Server", "rig_specs", "rig_frames", "arrivals", "run",
           "GpuExecutor", "BatchedGpuExecutor", "LearnedGpuExecutor", "latency_summary"]

RESOLUTIONS = [(640, 360), (1280, 720), (1920, 1080)]
RANGES = [64, 128, 256]


@dataclass(frozen=True)
class FrameSpec:
    width: int
    height: int
    num_disp: int


@dataclass
class Request:
    rid: int
    rig: int
    seq: int
    spec: FrameSpec
    left: object          # host image (uint8 [H][W]); pinned for the GPU executor
    right: object
    t_arrival: float
    deadline: float | None = None
    inject: str | None = None  # fault injection for tests: "launch" makes the launch of this request raise


@dataclass
class Result:
    rid: int
    rig: int
    seq: int
    ok: bool
    disp: object = None
    error: str | None = None
    t_arrival: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class SlotPool:
    """Device memory of in-flight frames, bounded by `budget` bytes. A slot belongs to one
    frame shape and is reused by later frames of that shape; idle slots of other shapes are
    freed (least recently used first) when a new one would not fit."""

    def __init__(self, budget: int, bytes_fn, alloc_fn, free_fn):
        self.budget = int(budget)
        self.bytes_fn, self.alloc_fn, self.free_fn = bytes_fn, alloc_fn, free_fn
        self.idle: OrderedDict[int, tuple] = OrderedDict()  # id -> (spec, slot, bytes)
        self.held = 0          # bytes of all slots, idle or busy
        self.busy = 0          # bytes of busy slots
        self.peak = 0
        self._next = 0

    def acquire(self, spec: FrameSpec):
        need = self.bytes_fn(spec)
        for k, (s, slot, b) in self.idle.items():
            if s == spec:
                del self.idle[k]
                self.busy += b
                return slot, b
        # free idle slots (other shapes) until the new one fits
        while self.held + need > self.budget and self.idle:
            _, (s, slot, b) = self.idle.popitem(last=False)
            self.free_fn(slot)
            self.held -= b
        if self.held + need > self.budget:
            return None
        slot = self.alloc_fn(spec)
        if slot is None:  # the executor has no slot of this shape free right now
            return None
        self.held += need
        self.busy += need
        self.peak = max(self.peak, self.held)
        return slot, need

    def release(self, spec: FrameSpec, slot, nbytes: int):
        self.busy -= nbytes
        self._next += 1
        self.idle[self._next] = (spec, slot, nbytes)

    def close(self):
        for _, (s, slot, b) in list(self.idle.items()):
            self.free_fn(slot)
            self.held -= b
        self.idle.clear()


class Server:
    """Admission queue + continuous batching over an executor."""

    def __init__(self, executor, budget: int, max_inflight: int = 16, max_batch: int = 8,
                 clock=time.perf_counter):
        self.ex = executor
        self.clock = clock
        self.pool = SlotPool(budget, executor.bytes_needed, executor.alloc, executor.free)
        self.max_inflight, self.max_batch = max_inflight, max_batch
        self.queue: deque[Request] = deque()
        self.inflight: list = []   # (ticket, request, slot, bytes, t_admit)
        self.results: list[Result] = []
        self.launches = 0
        self.batch_sizes: list[int] = []
        self.max_busy = 0

    def offer(self, req: Request):
        self.queue.append(req)

    def _fail(self, req: Request, why: str, now: float, t_admit: float = 0.0):
        self.results.append(Result(req.rid, req.rig, req.seq, False, None, why, req.t_arrival, t_admit, now))

    def pending(self) -> int:
        return len(self.queue) + len(self.inflight)

    def step(self):
        """Collect finished frames, then admit and launch what fits. Returns the number of
        frames completed in this step."""
        now = self.clock()
        done = 0
        still = []
        for item in self.inflight:
            ticket, req, slot, nb, t_admit = item
            if self.ex.done(ticket):
                out = self.ex.collect(ticket)
                t = self.clock()
                if isinstance(out, Exception):
                    self._fail(req, f"{type(out).__name__}: {out}", t, t_admit)
                else:
                    self.results.append(Result(req.rid, req.rig, req.seq, True, out, None, req.t_arrival, t_admit, t))
                self.pool.release(req.spec, slot, nb)
                done += 1
            else:
                still.append(item)
        self.inflight = still
        # admission: FIFO, the head waits until it fits
        batch = []
        now = self.clock()
        while self.queue and len(self.inflight) + len(batch) < self.max_inflight and len(batch) < self.max_batch:
            req = self.queue[0]
            if req.deadline is not None and now > req.deadline:
                self.queue.popleft()
                self._fail(req, "expired in queue", now)
                continue
            need = self.ex.bytes_needed(req.spec)
            if need <= 0:
                self.queue.popleft()
                self._fail(req, "invalid frame shape or disparity range", now)
                continue
            if need > self.pool.budget:
                self.queue.popleft()
                self._fail(req, "frame does not fit in the HBM budget", now)
                continue
            got = self.pool.acquire(req.spec)
            if got is None:
                break
            self.queue.popleft()
            batch.append((req, got[0], got[1]))
        self.max_busy = max(self.max_busy, self.pool.busy)
        if batch:
            tickets = self.ex.launch([(r, s) for r, s, _ in batch])
            t_admit = self.clock()
            self.launches += 1
            self.batch_sizes.append(len(batch))
            for (req, slot, nb), tk in zip(batch, tickets):
                self.inflight.append((tk, req, slot, nb, t_admit))
        return done

    def close(self):
        self.pool.close()


# ---------------------------------------------------------------------------------------
# Rigs and the driving loop
# ---------------------------------------------------------------------------------------
def rig_specs(n_rigs: int = 8, seed: int = 5):
    """Per-rig (resolution, disparity range), drawn by `seed`."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    res = rng.integers(0, len(RESOLUTIONS), n_rigs)
    rngs = rng.integers(0, len(RANGES), n_rigs)
    return [FrameSpec(*RESOLUTIONS[a], RANGES[b]) for a, b in zip(res, rngs)]


def rig_frames(specs, per_rig: int, seed: int = 5, workers: int = 16, pinned: bool = False):
    """Pre-generated frames of each rig (seeds seed*10^6 + rig*10^5 + f), cycled by the rigs."""
    from .scene import batch_scenes
    flat = [(seed * 10**6 + r * 10**5 + f, sp.width, sp.height, sp.num_disp, 30)
            for r, sp in enumerate(specs) for f in range(per_rig)]
    scenes = batch_scenes(flat, workers=workers)
    out = []
    for r in range(len(specs)):
        frames = []
        for sc in scenes[r * per_rig:(r + 1) * per_rig]:
            l, rr = sc.left, sc.right
            if pinned:
                import torch
                l = torch.from_numpy(l).pin_memory()
                rr = torch.from_numpy(rr).pin_memory()
            frames.append((l, rr))
        out.append(frames)
    return out


def arrivals(n_rigs: int, fps: float, duration: float, seed: int = 5, jitter: float = 1e-3):
    """Sorted (t, rig, seq): rig r delivers frame f at phase_r + f/fps + U(-jitter, jitter)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1])))
    out = []
    period = 1.0 / fps
    for r in range(n_rigs):
        phase = rng.uniform(0, period)
        n = int(np.floor((duration - phase) / period)) + 1 if duration > phase else 0
        t = phase + np.arange(n) * period + rng.uniform(-jitter, jitter, n)
        out += [(max(0.0, float(x)), r, f) for f, x in enumerate(t)]
    out.sort()
    return out


def run(server: Server, schedule, make_request, clock=time.perf_counter, wait=None, deadline_s=None):
    """Offers each scheduled frame at its time (relative to the start) and steps the server
    until every frame has a result. `wait(t)` idles until absolute clock time t (default:
    short sleeps); a virtual clock passes its own."""
    t0 = clock()
    i = 0
    n = len(schedule)
    rid = 0
    while i < n or server.pending():
        now = clock() - t0
        while i < n and schedule[i][0] <= now:
            t, rig, seq = schedule[i]
            req = make_request(rid, rig, seq, t0 + t)
            if deadline_s is not None:
                req.deadline = t0 + t + deadline_s
            server.offer(req)
            rid += 1
            i += 1
        server.step()
        nxt = t0 + schedule[i][0] if i < n else None
        if wait is not None:
            wait(nxt)
        elif server.inflight or nxt is None:
            time.sleep(0.0002)
        else:
            time.sleep(max(0.0, min(0.0005, nxt - clock())))
    return server.results


def latency_summary(results, t_span: float | None = None):
    ok = [r for r in results if r.ok]
    lat = np.array([r.latency * 1e3 for r in ok]) if ok else np.zeros(1)
    out = {"frames": len(results), "ok": len(ok), "failed": len(results) - len(ok),
           "p50_ms": round(float(np.percentile(lat, 50)), 4), "p99_ms": round(float(np.percentile(lat, 99)), 4),
           "max_ms": round(float(lat.max()), 4)}
    if t_span:
        out["frames_per_s"] = round(len(ok) / t_span, 1)
    return out


# ---------------------------------------------------------------------------------------
# GPU executor: one multi-scale matcher (HIP library) per slot
# ---------------------------------------------------------------------------------------
@dataclass
class _Slot:
    spec: FrameSpec
    left: object
    right: object
    matcher: object
    host_out: object
    event: object = None
    extra: dict = field(default_factory=dict)


class GpuExecutor:
    """Uploads, matches (multi-scale MPV, fixed +/-radius bands) and downloads each frame on
    one of `streams` HIP streams; a frame is done when its own event has completed."""

    def __init__(self, levels: int = 3, radius: int = 4, num_paths: int = 8, streams: int = 2,
                 device="cuda", sched=None):
        import torch
        from . import _lib
        _lib.lib()  # the HIP library is required; there is no other path
        self.torch = torch
        self.levels, self.radius, self.num_paths = levels, radius, num_paths
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.k = 0
        self.sched = sched
        self._bytes: dict = {}

    def params(self, spec: FrameSpec):
        from . import mpv
        return mpv.MPVParams(num_disp=spec.num_disp, num_paths=self.num_paths)

    def levels_for(self, spec: FrameSpec) -> int:
        return self.levels

    def bytes_needed(self, spec: FrameSpec) -> int:
        if spec in self._bytes:
            return self._bytes[spec]
        from . import mpv
        from ._lib import MPVError
        try:
            ws = mpv.pyramid_workspace_bytes(self.params(spec), self.levels_for(spec), self.radius,
                                             spec.width, spec.height, self.sched)
        except (MPVError, ValueError):
            ws = 0
        if ws <= 0:
            self._bytes[spec] = 0
            return 0
        W, H = spec.width, spec.height
        total = int(ws) + 2 * W * H + 3 * 2 * W * H  # workspace, both views, disp/raw/right maps
        self._bytes[spec] = total
        return total

    def alloc(self, spec: FrameSpec):
        from . import mpv
        torch = self.torch
        W, H = spec.width, spec.height
        m = mpv.Pyramid(self.params(spec), W, H, levels=self.levels_for(spec), radius=self.radius,
                        device=self.device, sched=self.sched)
        return _Slot(spec, torch.empty((H, W), dtype=torch.uint8, device=self.device),
                     torch.empty((H, W), dtype=torch.uint8, device=self.device), m,
                     torch.empty((H, W), dtype=torch.int16, pin_memory=True), torch.cuda.Event())

    def free(self, slot: _Slot):
        slot.matcher = None
        slot.left = slot.right = None

    def launch(self, items):
        torch = self.torch
        s = self.streams[self.k % len(self.streams)]
        self.k += 1
        tickets = []
        with torch.cuda.stream(s):
            for req, slot in items:
                try:
                    if req.inject == "launch":
                        raise RuntimeError("injected launch fault")
                    slot.left.copy_(req.left, non_blocking=True)
                    slot.right.copy_(req.right, non_blocking=True)
                    out = slot.matcher(slot.left, slot.right)
                    slot.host_out.copy_(out, non_blocking=True)
                    slot.event.record(s)
                    tickets.append(slot)
                except Exception as e:  # the failing request only
                    tickets.append(e)
        return tickets

    def done(self, ticket) -> bool:
        return isinstance(ticket, Exception) or ticket.event.query()

    def collect(self, ticket):
        if isinstance(ticket, Exception):
            return ticket
        return ticket.host_out.numpy().copy()


# ---------------------------------------------------------------------------------------
# Batched GPU executor: the frames admitted together run as one batched launch per stage
# ---------------------------------------------------------------------------------------
class _ArenaSlot:
    def __init__(self, idx, spec, left, right, host_out):
        self.idx, self.spec, self.left, self.right, self.host_out = idx, spec, left, right, host_out
        self.event = None


class BatchedGpuExecutor:
    """Continuous batching through the batched kernels: a fixed arena of `per_spec` slots per
    rig for each frame shape the rigs deliver (device inputs, outputs and workspace regions of one
    mpv_batch over all of them). The frames admitted in one scheduler step are uploaded on an
    upload stream and matched by one mpv_batch_run_items call (every stage one launch over
    those frames) on the compute stream, which waits for the uploads; the downloads run on a
    download stream behind the step's kernels and every frame of the step completes on the
    step's event. Uploads of the next step and downloads of the previous one overlap the
    current step's kernels. Each frame's result equals mpv_pyramid of that frame alone.
    Default schedule: the batched layouts (one line per lane for the banded levels' vertical and
    diagonal directions, longest lines first, two waves per block). Steps that admit at most
    `lone_max` frames (light load) run a second batch over the same slots with the lane-group
    layouts instead, whose chains are short: a lone frame's latency, where the batched layouts
    would turn its lines into long serial chains (0 = always the first batch)."""

    def __init__(self, specs, per_spec: int = 4, levels: int = 3, radius: int = 4, num_paths: int = 8,
                 device="cuda", sched=None, lone_max: int = 3, lone_sched=None):
        import torch
        from . import _lib, mpv
        _lib.lib()  # the HIP library is required; there is no other path
        self.torch = torch
        self.device = torch.device(device)
        self.levels, self.radius, self.num_paths = levels, radius, num_paths
        self.upload = torch.cuda.Stream(device=self.device)
        self.compute = torch.cuda.Stream(device=self.device)
        self.download = torch.cuda.Stream(device=self.device)
        uniq = []
        for sp in specs:
            if sp not in uniq and self._valid(sp):
                uniq.append(sp)
        self.slots, self.free_slots = [], {}
        pairs = []
        for sp in uniq:
            self.free_slots[sp] = []
            # per_spec slots for every rig delivering this shape, so that rigs sharing a shape
            # do not block the queue's head on each other's slots
            for _ in range(per_spec * sum(1 for x in specs if x == sp)):
                L = torch.zeros((sp.height, sp.width), dtype=torch.uint8, device=self.device)
                R = torch.zeros_like(L)
                host = torch.empty((sp.height, sp.width), dtype=torch.int16, pin_memory=True)
                slot = _ArenaSlot(len(self.slots), sp, L, R, host)
                self.slots.append(slot)
                self.free_slots[sp].append(slot)
                pairs.append((L, R, sp.num_disp))
        params = mpv.MPVParams(num_disp=max(sp.num_disp for sp in uniq), num_paths=num_paths)
        if sched is None:
            sched = mpv.Schedule(waves_per_block=2, band_lanes=mpv.Schedule.LINE, order=1)
        self.lone_max = lone_max
        self.launches = {"batched": 0, "lone": 0}  # admission steps run by each batch
        with torch.cuda.stream(self.compute):
            self.batch = mpv.Batch(pairs, params, levels, radius, sched=sched, device=self.device)
            self.lone = (mpv.Batch(pairs, params, levels, radius, sched=lone_sched or mpv.Schedule(waves_per_block=4),
                                   device=self.device) if lone_max > 0 else None)
        # a slot: both images (2 B per pixel) and each batch's int16 disparity output
        self.px_bytes = 2 + 2 * (2 if self.lone is not None else 1)
        self.arena_bytes = int(self.batch.workspace.numel()) + sum(
            self.px_bytes * s.spec.width * s.spec.height for s in self.slots)
        if self.lone is not None:
            self.arena_bytes += int(self.lone.workspace.numel())
        self._bytes = {}

    def _valid(self, spec) -> bool:
        from . import mpv
        from ._lib import MPVError
        try:
            ws = mpv.pyramid_workspace_bytes(mpv.MPVParams(num_disp=spec.num_disp, num_paths=self.num_paths),
                                             self.levels, self.radius, spec.width, spec.height)
        except (MPVError, ValueError):
            return False
        return ws > 0

    def bytes_needed(self, spec) -> int:
        """Bytes one in-flight frame of this shape occupies in the arena (0: not served)."""
        if spec in self._bytes:
            return self._bytes[spec]
        if spec not in self.free_slots:
            self._bytes[spec] = 0
            return 0
        from . import mpv
        ws = mpv.pyramid_workspace_bytes(mpv.MPVParams(num_disp=spec.num_disp, num_paths=self.num_paths),
                                         self.levels, self.radius, spec.width, spec.height)
        self._bytes[spec] = int(ws) + self.px_bytes * spec.width * spec.height
        return self._bytes[spec]

    def alloc(self, spec):
        free = self.free_slots.get(spec)
        return free.pop() if free else None

    def free(self, slot):
        self.free_slots[slot.spec].append(slot)

    def launch(self, items):
        torch = self.torch
        tickets, run = [], []
        with torch.cuda.stream(self.upload):
            for req, slot in items:
                try:
                    if req.inject == "launch":
                        raise RuntimeError("injected launch fault")
                    slot.left.copy_(req.left, non_blocking=True)
                    slot.right.copy_(req.right, non_blocking=True)
                    run.append(slot)
                    tickets.append(slot)
                except Exception as e:  # the failing request only
                    tickets.append(e)
            up = torch.cuda.Event()
            up.record(self.upload)
        if run:
            lone = self.lone is not None and len(run) <= self.lone_max
            b = self.lone if lone else self.batch
            self.launches["lone" if lone else "batched"] += 1
            with torch.cuda.stream(self.compute):
                self.compute.wait_event(up)
                b.run_items([s.idx for s in run])
                matched = torch.cuda.Event()
                matched.record(self.compute)
            with torch.cuda.stream(self.download):
                self.download.wait_event(matched)
                for slot in run:
                    slot.host_out.copy_(b.disp[slot.idx], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.download)
            for slot in run:
                slot.event = ev
        return tickets

    def done(self, ticket) -> bool:
        return isinstance(ticket, Exception) or ticket.event.query()

    def collect(self, ticket):
        if isinstance(ticket, Exception):
            return ticket
        return ticket.host_out.numpy().copy()

    def close(self):
        self.compute.synchronize()
        self.download.synchronize()
        self.batch.close()
        if self.lone is not None:
            self.lone.close()


# ---------------------------------------------------------------------------------------
# Learned-band executor: proposal, then the banded finest level or the plain fallback
# ---------------------------------------------------------------------------------------
class _LearnedTicket:
    def __init__(self, slot, stream):
        self.slot, self.stream, self.phase, self.event = slot, stream, 1, None


class LearnedGpuExecutor(GpuExecutor):
    """Frames matched by the learned-band path with plain fallback: the launch enqueues the
    upload and the proposal (coarse level, network, fine bands; the low-confidence count
    follows into pinned memory behind an event); once the scheduler sees that event complete
    it enqueues, on the same stream, the banded finest level, or plain full-range MPV for a
    frame whose low-confidence fraction is above the threshold, then the download. Nothing
    blocks the host; `fallback_fraction` counts the fallback frames."""

    def __init__(self, net, cfg=None, **kw):
        super().__init__(**kw)
        self.net, self.cfg = net, cfg
        self.frames = 0
        self.fallbacks = 0

    def bytes_needed(self, spec) -> int:
        if spec in self._bytes:
            return self._bytes[spec]
        from . import mpv
        from ._lib import MPVError
        p = self.params(spec)
        try:
            full = mpv.match_workspace_bytes(p, spec.width, spec.height)
        except (MPVError, ValueError):
            full = 0
        if full <= 0 or spec.width >> 2 < 1 or spec.height >> 2 < 1:
            self._bytes[spec] = 0
            return 0
        W, H = spec.width, spec.height
        # full-range workspace (fallback), bands, both views, maps and the coarse level's buffers
        total = int(full) + 3 * W * H + 2 * W * H + 2 * W * H + (W >> 2) * (H >> 2) * 64
        self._bytes[spec] = total
        return total

    def alloc(self, spec):
        from .learned import LearnedMatcher
        torch = self.torch
        W, H = spec.width, spec.height
        m = LearnedMatcher(self.net, self.params(spec), W, H, self.cfg, device=self.device)
        return _Slot(spec, torch.empty((H, W), dtype=torch.uint8, device=self.device),
                     torch.empty((H, W), dtype=torch.uint8, device=self.device), m,
                     torch.empty((H, W), dtype=torch.int16, pin_memory=True), torch.cuda.Event())

    def launch(self, items):
        torch = self.torch
        s = self.streams[self.k % len(self.streams)]
        self.k += 1
        tickets = []
        with torch.cuda.stream(s):
            for req, slot in items:
                try:
                    if req.inject == "launch":
                        raise RuntimeError("injected launch fault")
                    slot.left.copy_(req.left, non_blocking=True)
                    slot.right.copy_(req.right, non_blocking=True)
                    slot.matcher.propose(slot.left, slot.right)
                    tickets.append(_LearnedTicket(slot, s))
                except Exception as e:  # the failing request only
                    tickets.append(e)
        return tickets

    def done(self, ticket) -> bool:
        if isinstance(ticket, Exception):
            return True
        if ticket.phase == 1:
            m = ticket.slot.matcher
            if not m.ready():
                return False
            torch = self.torch
            fb = m.fallback_due()
            with torch.cuda.stream(ticket.stream):
                out = m.finish(ticket.slot.left, ticket.slot.right, fb)
                ticket.slot.host_out.copy_(out, non_blocking=True)
                ticket.slot.event.record(ticket.stream)
            self.frames += 1
            self.fallbacks += int(fb)
            ticket.phase = 2
            return False
        return ticket.slot.event.query()

    def collect(self, ticket):
        if isinstance(ticket, Exception):
            return ticket
        return ticket.slot.host_out.numpy().copy()

    @property
    def fallback_fraction(self):
        return self.fallbacks / self.frames if self.frames else None
