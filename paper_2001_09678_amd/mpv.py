"""Python face of the HIP MPV library: argument marshalling only.

Every step of the matcher runs in the HIP kernels of ``libmpv.so``; this module allocates
outputs and workspaces as torch tensors on the current device and passes their pointers
and ``torch.cuda.current_stream()`` through the C ABI of include/mpv.h. Tensors must be
CUDA (HIP) tensors; anything else is an error, never a fallback.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as _L


@dataclass(frozen=True)
class MPVParams:
    """Matcher parameters (eq. e(p,u) transition lambda*min(|d-d'|, tau); Table alg paths)."""
    num_disp: int = 64
    num_paths: int = 4
    lam: int = 8
    tau: int = 4
    lr_max_diff: int = 1
    agg_type: str = "u16"  # exported aggregate type: "u16" or "i32"
    # path merge: "sum", or the hierarchical merge of Section 3.2 (Table alg), "layered",
    # or "layered_occ" with its occlusion strategy
    merge: str = "sum"
    # 0: constant lambda; 1..255: gradient-weighted TV of eq. EU (lambda * e^(-|dI| / sigma))
    grad_sigma: int = 0
    # matching cost: "census" (Hamming of 5x5 census signatures) or "ssim" (Section 3.2)
    data_term: str = "census"

    _MERGES = {"sum": _L.MPV_MERGE_SUM, "layered": _L.MPV_MERGE_LAYERED,
               "layered_occ": _L.MPV_MERGE_LAYERED_OCC}

    def c(self) -> _L.Params:
        if self.merge not in self._MERGES:
            raise ValueError(f"merge must be one of {sorted(self._MERGES)}")
        if self.data_term not in ("census", "ssim"):
            raise ValueError("data_term must be 'census' or 'ssim'")
        return _L.Params(self.num_disp, 2, self.num_paths, self.lam, self.tau, self.lr_max_diff,
                         _L.MPV_AGG_U16 if self.agg_type == "u16" else _L.MPV_AGG_I32,
                         self._MERGES[self.merge], self.grad_sigma,
                         _L.MPV_DATA_SSIM if self.data_term == "ssim" else _L.MPV_DATA_CENSUS)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t


def _image(t: torch.Tensor, name: str) -> _L.Image:
    _dev(t, torch.uint8, name)
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D uint8 tensor with unit column stride")
    return _L.Image(t.data_ptr(), t.shape[1], t.shape[0], t.stride(0))


@dataclass
class Band:
    """Per-pixel search band: disparities lo .. lo+len-1 (len None: cap everywhere)."""
    lo: torch.Tensor           # int16 [H][W]
    cap: int
    length: torch.Tensor | None = None  # uint8 [H][W]

    def c(self) -> _L.Band:
        _dev(self.lo, torch.int16, "band.lo")
        ln = None
        if self.length is not None:
            ln = _dev(self.length, torch.uint8, "band.length").data_ptr()
        return _L.Band(self.lo.contiguous().data_ptr(), ln, self.cap)


def _band(band: Band | None):
    return None if band is None else C.byref(band.c())


def census(img: torch.Tensor) -> torch.Tensor:
    im = _image(img, "img")
    out = torch.empty((im.height, im.width), dtype=torch.int32, device=img.device)
    _L.check(_L.lib().mpv_census(C.byref(im), out.data_ptr(), _stream()), "mpv_census")
    return out


def downsample(img: torch.Tensor) -> torch.Tensor:
    im = _image(img, "img")
    out = torch.empty((im.height // 2, im.width // 2), dtype=torch.uint8, device=img.device)
    _L.check(_L.lib().mpv_downsample(C.byref(im), out.data_ptr(), _stream()), "mpv_downsample")
    return out


def cost(left: torch.Tensor, right: torch.Tensor, params: MPVParams, band: Band | None = None):
    li, ri = _image(left, "left"), _image(right, "right")
    cap = params.num_disp if band is None else band.cap
    out = torch.empty((li.height, li.width, cap), dtype=torch.uint8, device=left.device)
    p = params.c()
    _L.check(_L.lib().mpv_cost(C.byref(p), C.byref(li), C.byref(ri), _band(band), out.data_ptr(),
                               _stream()), "mpv_cost")
    return out


def aggregate(cost_vol: torch.Tensor, params: MPVParams, band: Band | None = None,
              path_mask: int = 0) -> torch.Tensor:
    """Unnormalised sum of the selected path energies. uint16 sums are returned in an
    int16 tensor holding the same bits (view as uint16 to read them)."""
    _dev(cost_vol, torch.uint8, "cost")
    cost_vol = cost_vol.contiguous()
    h, w, cap = cost_vol.shape
    dt = torch.int16 if params.agg_type == "u16" else torch.int32
    out = torch.empty((h, w, cap), dtype=dt, device=cost_vol.device)
    p = params.c()
    _L.check(_L.lib().mpv_aggregate(C.byref(p), cost_vol.data_ptr(), w, h, _band(band), path_mask,
                                    out.data_ptr(), _stream()), "mpv_aggregate")
    return out


def disparity(agg: torch.Tensor, params: MPVParams, band: Band | None = None):
    """WTA + right disparity + LR check on an aggregate volume. Returns (disp, right, raw)."""
    want = torch.int16 if params.agg_type == "u16" else torch.int32
    _dev(agg, want, "agg")
    agg = agg.contiguous()
    h, w, _ = agg.shape
    outs = [torch.empty((h, w), dtype=torch.int16, device=agg.device) for _ in range(3)]
    p = params.c()
    _L.check(_L.lib().mpv_disparity(C.byref(p), agg.data_ptr(), w, h, _band(band),
                                    outs[0].data_ptr(), outs[1].data_ptr(), outs[2].data_ptr(),
                                    _stream()), "mpv_disparity")
    return tuple(outs)


def match_workspace_bytes(params: MPVParams, width: int, height: int, band: Band | None = None) -> int:
    p = params.c()
    return int(_L.lib().mpv_match_workspace_bytes(C.byref(p), width, height, _band(band)))


def match(left, right, params: MPVParams, band: Band | None = None, workspace=None, want_all=False):
    """One fused level (cost -> all paths -> sum -> WTA -> LR)."""
    li, ri = _image(left, "left"), _image(right, "right")
    need = match_workspace_bytes(params, li.width, li.height, band)
    if need == 0:
        raise _L.MPVError(_L.MPV_ERR_INVALID_ARG, "mpv_match_workspace_bytes")
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=left.device)
    disp = torch.empty((li.height, li.width), dtype=torch.int16, device=left.device)
    right_d = torch.empty_like(disp) if want_all else None
    raw = torch.empty_like(disp) if want_all else None
    p = params.c()
    _L.check(_L.lib().mpv_match(C.byref(p), C.byref(li), C.byref(ri), _band(band), disp.data_ptr(),
                                None if right_d is None else right_d.data_ptr(),
                                None if raw is None else raw.data_ptr(),
                                workspace.data_ptr(), workspace.numel(), _stream()), "mpv_match")
    return (disp, right_d, raw) if want_all else disp


@dataclass(frozen=True)
class Schedule:
    """Launch schedule (all give bit-identical results): waves per scan block (1/2/4),
    lanes per line of full-range scans (0 default, 16/32/64), lanes per line of banded
    scans (0 default, 16/32/64, or 1 = ``LINE``: one line per lane for the vertical and
    diagonal directions where the level allows it), batched scan order (0 pair by pair,
    1 longest first)."""
    LINE = _L.MPV_BAND_LANES_LINE
    waves_per_block: int = 0
    full_lanes: int = 0
    band_lanes: int = 0
    order: int = 0

    def c(self) -> _L.Schedule:
        return _L.Schedule(self.waves_per_block, self.full_lanes, self.band_lanes, self.order)


_PROPAGATIONS = {"nearest": _L.MPV_PROP_NEAREST, "paper": _L.MPV_PROP_PAPER}


def pyramid_params(params: MPVParams, levels: int, radius: int, sched: Schedule | None = None,
                   propagation: str = "nearest", block: int = 0) -> _L.PyramidParams:
    """``propagation`` "nearest" (bands centred on twice the parent's raw winner) or "paper"
    (Section 3.4: block modes at intermediate levels, ``block`` pixels at level 1 (0 = 8),
    linear interpolation at the last level)."""
    if propagation not in _PROPAGATIONS:
        raise ValueError(f"propagation must be one of {sorted(_PROPAGATIONS)}")
    return _L.PyramidParams(params.c(), levels, radius, (sched or Schedule()).c(), _PROPAGATIONS[propagation],
                            block)


def pyramid_workspace_bytes(params: MPVParams, levels: int, radius: int, width: int, height: int,
                            sched: Schedule | None = None, propagation: str = "nearest", block: int = 0) -> int:
    pp = pyramid_params(params, levels, radius, sched, propagation, block)
    return int(_L.lib().mpv_pyramid_workspace_bytes(C.byref(pp), width, height))


class Pyramid:
    """Multi-scale MPV (Section 3.4) on one pair shape, with its workspace held for reuse.

    ``levels=1`` is plain single-scale MPV. Calling the object enqueues the whole path on the
    current stream and returns the finest LR-checked disparity (int16, -1 invalid)."""

    def __init__(self, params: MPVParams, width: int, height: int, levels: int = 3, radius: int = 4,
                 device="cuda", keep_levels: bool = False, sched: Schedule | None = None,
                 propagation: str = "nearest", block: int = 0):
        self.params, self.width, self.height = params, width, height
        self.levels, self.radius = levels, radius
        self._pp = pyramid_params(params, levels, radius, sched, propagation, block)
        need = int(_L.lib().mpv_pyramid_workspace_bytes(C.byref(self._pp), width, height))
        if need == 0:
            raise _L.MPVError(_L.MPV_ERR_INVALID_ARG, "mpv_pyramid_workspace_bytes")
        self.workspace = torch.empty(need, dtype=torch.uint8, device=device)
        self.disp = torch.empty((height, width), dtype=torch.int16, device=device)
        self.raw = torch.empty_like(self.disp)
        self.right = torch.empty_like(self.disp)
        self.level_raw = []
        if keep_levels:
            for l in range(levels):
                s = levels - 1 - l
                self.level_raw.append(torch.empty((height >> s, width >> s), dtype=torch.int16, device=device))
        self._out = _L.PyramidOut(self.disp.data_ptr(), self.raw.data_ptr(), self.right.data_ptr())
        for l, t in enumerate(self.level_raw):
            self._out.level_raw[l] = t.data_ptr()

    def __call__(self, left: torch.Tensor, right: torch.Tensor) -> torch.Tensor:
        li, ri = _image(left, "left"), _image(right, "right")
        if (li.width, li.height) != (self.width, self.height):
            raise ValueError("pair shape differs from the shape this Pyramid was built for")
        _L.check(_L.lib().mpv_pyramid(C.byref(self._pp), C.byref(li), C.byref(ri), C.byref(self._out),
                                      self.workspace.data_ptr(), self.workspace.numel(), _stream()),
                 "mpv_pyramid")
        return self.disp


def pyramid(left, right, params: MPVParams, levels=3, radius=4, keep_levels=False, sched=None,
            propagation="nearest", block=0):
    h, w = left.shape
    pyr = Pyramid(params, w, h, levels, radius, device=left.device, keep_levels=keep_levels, sched=sched,
                  propagation=propagation, block=block)
    pyr(left, right)
    return pyr


class Batch:
    """Many stereo pairs of different sizes and ranges matched together: every stage of
    every pyramid level is one launch over all pairs (descriptor table in the workspace),
    optionally replayed as one captured hipGraph. Each pair's output equals its solo
    mpv_pyramid result. The pairs' input tensors are held by reference; refill them in
    place between runs (``run`` reads whatever they hold)."""

    def __init__(self, pairs, params: MPVParams, levels=3, radius=4, sched: Schedule | None = None,
                 device="cuda", want_all=False):
        self.params, self.levels, self.radius = params, levels, radius
        self.sched = sched if sched is not None else Schedule()
        self.pairs = list(pairs)  # [(left, right, num_disp)]
        self.disp, self.right, self.raw = [], [], []
        items = (_L.BatchItem * len(self.pairs))()
        for i, (l, r, d) in enumerate(self.pairs):
            li, ri = _image(l, f"left[{i}]"), _image(r, f"right[{i}]")
            out = torch.empty(l.shape, dtype=torch.int16, device=l.device)
            rt = torch.empty_like(out) if want_all else None
            rw = torch.empty_like(out) if want_all else None
            self.disp.append(out)
            self.right.append(rt)
            self.raw.append(rw)
            items[i] = _L.BatchItem(li, ri, int(d), out.data_ptr(),
                                    None if rt is None else rt.data_ptr(),
                                    None if rw is None else rw.data_ptr())
        pp = pyramid_params(params, levels, radius, sched)
        h = C.c_void_p()
        _L.check(_L.lib().mpv_batch_create(C.byref(pp), items, len(self.pairs), C.byref(h)),
                 "mpv_batch_create")
        self._h = h
        need = int(_L.lib().mpv_batch_workspace_bytes(h))
        self.workspace = torch.empty(need, dtype=torch.uint8, device=device)
        _L.check(_L.lib().mpv_batch_bind(h, self.workspace.data_ptr(), need, _stream()),
                 "mpv_batch_bind")

    def run(self):
        _L.check(_L.lib().mpv_batch_run(self._h, _stream()), "mpv_batch_run")
        return self.disp

    def run_graph(self):
        _L.check(_L.lib().mpv_batch_run_graph(self._h, _stream()), "mpv_batch_run_graph")
        return self.disp

    def run_items(self, idx):
        """Match only the pairs idx (distinct indices) in one batched launch per stage."""
        arr = (C.c_int32 * len(idx))(*[int(i) for i in idx])
        _L.check(_L.lib().mpv_batch_run_items(self._h, arr, len(idx), _stream()), "mpv_batch_run_items")
        return [self.disp[i] for i in idx]

    def close(self):
        if getattr(self, "_h", None):
            _L.lib().mpv_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vdisparity(disp: torch.Tensor, num_disp: int) -> torch.Tensor:
    """v-disparity image of a disparity map (Section 3.5, eq. disp_map): [D][H] counts of
    each row's disparities, as an int32 tensor holding the library's uint32 counts."""
    d = _dev(disp, torch.int16, "disp")
    if d.dim() != 2 or d.stride(1) != 1:
        raise ValueError("disp must be a 2-D map with contiguous rows")
    h, w = d.shape
    hist = torch.empty((num_disp, h), dtype=torch.int32, device=d.device)
    _L.check(_L.lib().mpv_vdisparity(d.data_ptr(), w, h, d.stride(0), num_disp, hist.data_ptr(), _stream()),
             "mpv_vdisparity")
    return hist


def udisparity(disp: torch.Tensor, num_disp: int) -> torch.Tensor:
    """u-disparity image of a disparity map (Section 3.5, eq. hy): [D][W] counts of each
    column's disparities, as an int32 tensor holding the library's uint32 counts."""
    d = _dev(disp, torch.int16, "disp")
    if d.dim() != 2 or d.stride(1) != 1:
        raise ValueError("disp must be a 2-D map with contiguous rows")
    h, w = d.shape
    hist = torch.empty((num_disp, w), dtype=torch.int32, device=d.device)
    _L.check(_L.lib().mpv_udisparity(d.data_ptr(), w, h, d.stride(0), num_disp, hist.data_ptr(), _stream()),
             "mpv_udisparity")
    return hist


def road(hist: torch.Tensor, eta: int = 8):
    """Road profile over a v-disparity image (Section 3.5, eqs. P_hat and e): the row of the
    road at every disparity (int16 [D], -1 if none) and the profile's sum of counts (int32 [1])."""
    h = _dev(hist, torch.int32, "hist")
    if h.dim() != 2 or not h.is_contiguous():
        raise ValueError("hist must be a contiguous [D][H] tensor")
    D, H = h.shape
    need = int(_L.lib().mpv_road_workspace_bytes(D, H))
    if need == 0:
        raise _L.MPVError(_L.MPV_ERR_INVALID_ARG, "mpv_road_workspace_bytes")
    ws = torch.empty(need, dtype=torch.uint8, device=h.device)
    path = torch.empty(D, dtype=torch.int16, device=h.device)
    energy = torch.empty(1, dtype=torch.int32, device=h.device)
    _L.check(_L.lib().mpv_road(h.data_ptr(), D, H, eta, path.data_ptr(), energy.data_ptr(), ws.data_ptr(),
                               need, _stream()), "mpv_road")
    return path, energy
