"""Schedule autotuner for the fused MPV path.

A schedule (waves per scan block, lanes per line of full-range and banded scans, order of
batched scans) changes only how work is laid out on the GPU, never a result: the tuner
times every candidate with HIP events on the current stream, checks that each candidate's
output is bit-identical to the default schedule's, and keeps the fastest. Results are
cached as JSON keyed by device architecture and workload.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os

import torch

from . import mpv

CACHE = os.environ.get("MPV_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "mpv", "tune.json"))


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _load() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def candidates(batched: bool = False):
    """Every schedule the tuner tries (all valid for any workload: a layout that does not
    fit a range falls back to the default layout inside the library)."""
    orders = (0, 1) if batched else (0,)
    # one line per lane pays off only with many frames in flight (a lone frame's lines are
    # long serial chains), so only batches try it
    bands = (0, 32, mpv.Schedule.LINE) if batched else (0, 32)
    out = []
    for wpb, fl, bl, order in itertools.product((1, 2, 4), (0, 32), bands, orders):
        out.append(mpv.Schedule(waves_per_block=wpb, full_lanes=fl, band_lanes=bl, order=order))
    return out


def _time(fn, reps: int, warmup: int = 3) -> float:
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_pyramid(left, right, params: mpv.MPVParams, levels: int, radius: int, reps: int = 20,
                 use_cache: bool = True, verbose: bool = False):
    """Fastest schedule for one pair shape; returns (schedule, {schedule: ms})."""
    h, w = left.shape
    key = f"{_arch()}|pyr|{w}x{h}|D{params.num_disp}|P{params.num_paths}|L{levels}|R{radius}|" \
          f"lam{params.lam}|tau{params.tau}|{params.merge}|g{params.grad_sigma}"
    cache = _load() if use_cache else {}
    if key in cache:
        return mpv.Schedule(**cache[key]["best"]), cache[key]["ms"]
    ref = mpv.pyramid(left, right, params, levels, radius)
    ref_bits = ref.disp.clone()
    times = {}
    for s in candidates():
        pyr = mpv.Pyramid(params, w, h, levels, radius, device=left.device, sched=s)
        ms = _time(lambda: pyr(left, right), reps)
        if not torch.equal(pyr.disp, ref_bits):
            raise AssertionError(f"schedule {s} changed the result")
        times[s] = ms
        if verbose:
            print(f"  {s}: {ms:.4f} ms", flush=True)
    best = min(times, key=times.get)
    if use_cache:
        cache[key] = {"best": best.__dict__, "ms": {str(k.__dict__): v for k, v in times.items()}}
        _store(cache)
    return best, times


def tune_batch(pairs, params: mpv.MPVParams, levels: int, radius: int, reps: int = 5,
               use_cache: bool = True, verbose: bool = False, key_extra: str = ""):
    """Fastest schedule for a batch of pairs (graph replay); returns (schedule, {schedule: ms})."""
    shapes = ",".join(f"{l.shape[1]}x{l.shape[0]}D{d}" for l, _, d in pairs)
    digest = hashlib.md5(shapes.encode()).hexdigest()[:12]
    key = f"{_arch()}|batch|{len(pairs)}|{digest}|P{params.num_paths}|L{levels}|" \
          f"R{radius}|lam{params.lam}|tau{params.tau}|{params.merge}|g{params.grad_sigma}{key_extra}"
    cache = _load() if use_cache else {}
    if key in cache:
        return mpv.Schedule(**cache[key]["best"]), cache[key]["ms"]
    ref = mpv.Batch(pairs, params, levels, radius)
    ref.run()
    ref_bits = [t.clone() for t in ref.disp]
    ref.close()
    times = {}
    for s in candidates(batched=True):
        b = mpv.Batch(pairs, params, levels, radius, sched=s)
        ms = _time(b.run_graph, reps)
        if any(not torch.equal(x, y) for x, y in zip(b.disp, ref_bits)):
            raise AssertionError(f"schedule {s} changed the result")
        times[s] = ms
        b.close()
        del b
        if verbose:
            print(f"  {s}: {ms:.3f} ms", flush=True)
    best = min(times, key=times.get)
    if use_cache:
        cache[key] = {"best": best.__dict__, "ms": {str(k.__dict__): v for k, v in times.items()}}
        _store(cache)
    return best, times
