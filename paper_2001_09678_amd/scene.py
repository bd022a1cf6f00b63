"""Seeded synthetic stereo scenes: the input producer shared by the GPU path and the oracle.

This module holds none of the matcher's arithmetic. It only draws images, so that every
test, benchmark and training run feeds identical bytes to the HIP library and to the CPU
oracle.

Scene model (the paper's plane geometry, Section 3.2, eqs. P/uxy/5): a world plane
ax+by+cz=1 seen by a rectified pair has a disparity that is an affine function of the
image coordinates, and the ground plane y=y0 gives a disparity that grows linearly with
the image row below the horizon. A scene is therefore built from

* a value-noise texture (lattice periods 32/16/8/4 px, amplitudes 1, 1/2, 1/4, 1/8,
  smoothstep-bilinear interpolation of uniform lattice values) mapped to [16, 239];
* K slanted disparity planes d = c + a(x-x0) + b(y-y0), one per Voronoi cell of K
  uniform seeds, c ~ U[0, dmax], a, b ~ U[-0.05, 0.05];
* optionally a ground ramp below the horizon y_h = H/2 with d_g(y) = 0.8 dmax (y-y_h)/(H-y_h),
  which a plane replaces only where the plane's disparity is larger;
* a right view made by forward-warping the left view: left (x, y) lands on right
  (x - d, y); a z-buffer keeps the larger disparity; pixels nothing lands on get
  fresh value noise from an independent stream; then N(0, sigma^2) noise, rounded to
  nearest and clamped to [0, 255], is added to the right view only.

Randomness: numpy's PCG64 generator, one independent child stream per purpose spawned
from ``numpy.random.SeedSequence(seed)``, so a seed fixes every byte of the scene.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = ["Scene", "make_scene", "value_noise", "constant_warp_pair", "config_scene"]


@dataclass
class Scene:
    left: np.ndarray      # uint8 [H][W]
    right: np.ndarray     # uint8 [H][W]
    disp: np.ndarray      # int16 [H][W], ground-truth disparity of the left view
    occluded: np.ndarray  # bool  [H][W], left pixels with no visible match in the right view


def _smoothstep(t: np.ndarray) -> np.ndarray:
    return t * t * (3.0 - 2.0 * t)


def value_noise(rng: np.random.Generator, height: int, width: int,
                periods=(32, 16, 8, 4), amplitudes=(1.0, 0.5, 0.25, 0.125)) -> np.ndarray:
    """Multi-octave value noise mapped to uint8 in [16, 239]."""
    acc = np.zeros((height, width), dtype=np.float64)
    ys = np.arange(height, dtype=np.float64)
    xs = np.arange(width, dtype=np.float64)
    for period, amp in zip(periods, amplitudes):
        gh = height // period + 2
        gw = width // period + 2
        lattice = rng.random((gh, gw))
        fy = ys / period
        fx = xs / period
        iy = np.floor(fy).astype(np.int64)
        ix = np.floor(fx).astype(np.int64)
        ty = _smoothstep(fy - iy)[:, None]
        tx = _smoothstep(fx - ix)[None, :]
        v00 = lattice[iy][:, ix]
        v01 = lattice[iy][:, ix + 1]
        v10 = lattice[iy + 1][:, ix]
        v11 = lattice[iy + 1][:, ix + 1]
        top = v00 + (v01 - v00) * tx
        bot = v10 + (v11 - v10) * tx
        acc += amp * (top + (bot - top) * ty)
    lo, hi = acc.min(), acc.max()
    if hi <= lo:
        return np.full((height, width), 128, dtype=np.uint8)
    img = 16.0 + (acc - lo) * (223.0 / (hi - lo))
    return np.clip(np.floor(img + 0.5), 16, 239).astype(np.uint8)


def _disparity_map(rng: np.random.Generator, height: int, width: int, dmax: int,
                   n_planes: int, ground: bool) -> np.ndarray:
    seeds_x = rng.random(n_planes) * width
    seeds_y = rng.random(n_planes) * height
    c = rng.random(n_planes) * dmax
    a = rng.uniform(-0.05, 0.05, n_planes)
    b = rng.uniform(-0.05, 0.05, n_planes)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64)
    best = np.full((height, width), np.inf)
    owner = np.zeros((height, width), dtype=np.int64)
    for k in range(n_planes):
        dist = (xx - seeds_x[k]) ** 2 + (yy - seeds_y[k]) ** 2
        closer = dist < best
        best[closer] = dist[closer]
        owner[closer] = k
    d = c[owner] + a[owner] * (xx - seeds_x[owner]) + b[owner] * (yy - seeds_y[owner])
    if ground:
        yh = height / 2.0
        dg = np.where(yy >= yh, 0.8 * dmax * (yy - yh) / max(height - yh, 1.0), -np.inf)
        d = np.maximum(d, dg)
    d = np.clip(d, 0.0, float(dmax))
    return np.floor(d + 0.5).astype(np.int16)


def make_scene(seed: int, width: int, height: int, dmax: int, n_planes: int,
               ground: bool = False, sigma: float = 2.0) -> Scene:
    """Piecewise-planar scene; ``dmax`` is the largest ground-truth disparity."""
    ss = np.random.SeedSequence(seed)
    s_tex, s_disp, s_hole, s_noise = (np.random.Generator(np.random.PCG64(c)) for c in ss.spawn(4))
    left = value_noise(s_tex, height, width)
    disp = _disparity_map(s_disp, height, width, dmax, n_planes, ground)
    right, occluded = _forward_warp(left, disp, value_noise(s_hole, height, width))
    if sigma > 0:
        noise = s_noise.normal(0.0, sigma, size=right.shape)
        right = np.clip(np.floor(right.astype(np.float64) + noise + 0.5), 0, 255).astype(np.uint8)
    return Scene(left=left, right=right, disp=disp, occluded=occluded)


def _forward_warp(left: np.ndarray, disp: np.ndarray, fill: np.ndarray):
    """Right view by forward warping the left view along rows; the larger disparity wins."""
    height, width = left.shape
    xs = np.broadcast_to(np.arange(width, dtype=np.int64), (height, width))
    ys = np.broadcast_to(np.arange(height, dtype=np.int64)[:, None], (height, width))
    d = disp.astype(np.int64)
    xt = xs - d
    inside = xt >= 0
    key = d * width + xs                                  # unique per source pixel of a row
    zbuf = np.full(height * width, -1, dtype=np.int64)
    tgt = (ys * width + xt)[inside]
    np.maximum.at(zbuf, tgt, key[inside])
    right = fill.copy().reshape(-1)
    hit = zbuf >= 0
    src_x = zbuf[hit] % width
    src_y = np.nonzero(hit)[0] // width
    right[hit] = left[src_y, src_x]
    visible = np.zeros((height, width), dtype=bool)
    visible[inside] = zbuf[tgt] == key[inside]
    return right.reshape(height, width), ~visible


def constant_warp_pair(seed: int, width: int, height: int, d0: int):
    """Left view of i.i.d. uniform noise; right(x, y) = left(x + d0, y), last d0 columns fresh noise.

    No added noise, so every interior pixel has an exact census match at disparity d0.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    left = rng.integers(0, 256, size=(height, width), dtype=np.uint8)
    right = rng.integers(0, 256, size=(height, width), dtype=np.uint8)
    if d0 < width:
        right[:, : width - d0] = left[:, d0:]
    return left, right


# Workloads: shapes and scene parameters of the configurations the library is measured on.
CONFIGS = {
    # plain single-scale MPV, 320x240, D=64, 4 paths, uint16 sums
    "c1": dict(width=320, height=240, num_disp=64, num_paths=4, levels=1, ground=False,
               planes=(6, 10), seed=1),
    # multi-scale MPV, 1280x720, D=128, 3 levels, +/-4 bands, 8 paths, int32 sums
    "c2": dict(width=1280, height=720, num_disp=128, num_paths=8, levels=3, ground=True,
               planes=(20, 40), seed=2),
    # the same pair matched at full range on one level (plain MPV at 1280x720, D=128)
    "c2p": dict(width=1280, height=720, num_disp=128, num_paths=8, levels=1, ground=True,
                planes=(20, 40), seed=2),
}


def config_scene(name: str, seed: int | None = None) -> tuple[Scene, dict]:
    cfg = dict(CONFIGS[name])
    s = cfg["seed"] if seed is None else seed
    lo, hi = cfg["planes"]
    k = lo + int(np.random.Generator(np.random.PCG64(np.random.SeedSequence([s, 7]))).integers(0, hi - lo + 1))
    scene = make_scene(s, cfg["width"], cfg["height"], cfg["num_disp"] - 1, k, ground=cfg["ground"])
    return scene, cfg


def config_specs(name: str, n: int) -> list[tuple]:
    """Specs (scene seed, width, height, D, planes) of n frames of a workload with a ground
    ramp: frame i is config_scene(name, seed + i), so frame 0 is the workload's own pair."""
    cfg = CONFIGS[name]
    assert cfg["ground"], "frames of a spec list carry the ground ramp"
    lo, hi = cfg["planes"]
    out = []
    for i in range(n):
        s = cfg["seed"] + i
        k = lo + int(np.random.Generator(np.random.PCG64(np.random.SeedSequence([s, 7]))).integers(0, hi - lo + 1))
        out.append((s, cfg["width"], cfg["height"], cfg["num_disp"], k))
    return out


# Batched workload: 64 pairs, sizes and ranges drawn uniformly (seed 3), pair i from seed 3000+i.
BATCH_SIZES = [(640, 360), (1280, 720), (1920, 1080)]
BATCH_DISPS = [64, 128, 256]


def batch_specs(n: int = 64, seed: int = 3):
    """(scene seed, width, height, D, planes) of each pair of the batched workload."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    sizes = rng.integers(0, len(BATCH_SIZES), n)
    disps = rng.integers(0, len(BATCH_DISPS), n)
    planes = rng.integers(20, 41, n)
    return [(seed * 1000 + i, *BATCH_SIZES[int(s)], BATCH_DISPS[int(d)], int(k))
            for i, (s, d, k) in enumerate(zip(sizes, disps, planes))]


def _spec_scene(spec):
    s, w, h, d, k = spec
    return make_scene(s, w, h, d - 1, k, ground=True)


def scene_chunks(specs, workers: int = 0, chunk: int = 64):
    """Yields the scenes of `specs` in order, `chunk` at a time (bounded host memory)."""
    if workers <= 1:
        for i in range(0, len(specs), chunk):
            yield [_spec_scene(sp) for sp in specs[i:i + chunk]]
        return
    import concurrent.futures as cf
    with cf.ProcessPoolExecutor(min(workers, len(specs))) as ex:
        pending = [ex.submit(_spec_scene, sp) for sp in specs[:chunk]]
        for i in range(0, len(specs), chunk):
            nxt = [ex.submit(_spec_scene, sp) for sp in specs[i + chunk:i + 2 * chunk]]
            yield [f.result() for f in pending]
            pending = nxt


def batch_scenes(specs, workers: int = 0):
    """Scenes of a list of specs, generated in parallel worker processes."""
    if workers <= 1 or len(specs) <= 1:
        return [_spec_scene(sp) for sp in specs]
    import concurrent.futures as cf
    with cf.ProcessPoolExecutor(min(workers, len(specs))) as ex:
        return list(ex.map(_spec_scene, specs))
