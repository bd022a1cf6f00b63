"""Learned band proposal: network, training and the learned-band matcher.

The network (five 3x3 convolutions, 8 -> 32 -> 32 -> 32 -> 32 -> 3, ReLU between) reads 8
features of the coarsest pyramid level (include/mpv_lb.h) and predicts per coarse pixel a
band center (offset to 4x the coarse winner), a band width (2..16) and a confidence. The
finest level then searches only that band; a coarse pixel below the confidence threshold
gets the widest band (16), and a frame with too many such pixels falls back to plain
full-range MPV. Every arithmetic step runs in the HIP kernels of libmpv.so (BF16 operands
with FP32 accumulation on MFMA for the convolutions); this module holds buffers, the data
pipeline and the training loop. Weights are trained on the GPU against labels produced by
plain full-range MPV on seeded synthetic scenes.
"""
from __future__ import annotations

import ctypes as C
import io
import json
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as _L
from . import mpv

CHANNELS = [8, 32, 32, 32, 32, 3]
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "bandnet.npz")


def _s():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class BandNet:
    """Parameters live in one flat FP32 buffer (per layer: w[3][3][cin][cout] then b[cout]);
    gradients and Adam moments use the same layout."""

    def __init__(self, device="cuda", seed: int = 0, params: np.ndarray | None = None):
        self.device = torch.device(device)
        self.layers = list(zip(CHANNELS[:-1], CHANNELS[1:]))
        self.offsets = []
        off = 0
        for cin, cout in self.layers:
            self.offsets.append((off, off + 9 * cin * cout))
            off += 9 * cin * cout + cout
        self.size = off
        if params is None:
            rng = np.random.default_rng(seed)
            params = np.zeros(self.size, np.float32)
            for (cin, cout), (wo, bo) in zip(self.layers, self.offsets):
                params[wo:bo] = rng.normal(0.0, np.sqrt(2.0 / (9 * cin)), 9 * cin * cout)
            # start the heads inside their linear ranges: width ~ 8, confidence ~ 0.5
            wo, bo = self.offsets[-1]
            params[bo + 1] = 6.0
            params[bo + 2] = 0.5
        self.params = torch.from_numpy(np.ascontiguousarray(params, np.float32)).to(self.device)
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        lib = _L.lib()
        self.wf = [torch.empty(int(lib.mpv_lb_packed_elems(ci, co)), dtype=torch.int16, device=self.device)
                   for ci, co in self.layers]
        self.wb = [torch.empty(int(lib.mpv_lb_packed_bwd_elems(ci, co)), dtype=torch.int16, device=self.device)
                   for ci, co in self.layers]
        self.pack()

    def w(self, i):
        wo, bo = self.offsets[i]
        return self.params[wo:bo]

    def b(self, i):
        _, bo = self.offsets[i]
        return self.params[bo:bo + self.layers[i][1]]

    def pack(self):
        lib = _L.lib()
        for i, (ci, co) in enumerate(self.layers):
            _L.check(lib.mpv_lb_pack(_p(self.w(i)), ci, co, _p(self.wf[i]), _p(self.wb[i]), _s()), "mpv_lb_pack")

    def forward(self, feat: torch.Tensor):
        """feat: bf16 bits (int16) [n][h][w][8]. Returns (o fp32 [n][h][w][4], activations)."""
        n, h, w, _ = feat.shape
        lib = _L.lib()
        acts = [feat]
        for i, (ci, co) in enumerate(self.layers):
            last = i + 1 == len(self.layers)
            y = torch.empty((n, h, w, 4 if last else co), dtype=torch.float32 if last else torch.int16,
                            device=self.device)
            _L.check(lib.mpv_lb_conv(_p(acts[-1]), n, h, w, ci, _p(self.wf[i]), _p(self.b(i)), co,
                                     0 if last else 1, None, 0, _p(y), y.shape[-1], 1 if last else 0, _s()),
                     "mpv_lb_conv")
            acts.append(y)
        return acts[-1], acts

    def backward(self, acts, dz_last: torch.Tensor, workspace: torch.Tensor | None = None):
        """dz_last: bf16 bits [n][h][w][4] (dL/do). Fills self.grad."""
        lib = _L.lib()
        n, h, w, _ = acts[0].shape
        need = max(int(lib.mpv_lb_dw_workspace_bytes(n, h, w, ci, co)) for ci, co in self.layers)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(need, dtype=torch.uint8, device=self.device)
        dz, dzs = dz_last, 4
        for i in range(len(self.layers) - 1, -1, -1):
            ci, co = self.layers[i]
            wo, bo = self.offsets[i]
            _L.check(lib.mpv_lb_conv_dw(_p(acts[i]), _p(dz), dzs, n, h, w, ci, co, _p(self.grad[wo:bo]),
                                        _p(self.grad[bo:bo + co]), _p(workspace), workspace.numel(), _s()),
                     "mpv_lb_conv_dw")
            if i == 0:
                break
            # dL/d(input of layer i) = conv with mirrored weights, times [activation > 0]
            nxt = torch.empty((n, h, w, ci), dtype=torch.int16, device=self.device)
            c4 = (co + 3) // 4 * 4
            _L.check(lib.mpv_lb_conv(_p(dz), n, h, w, c4, _p(self.wb[i]), None, ci, 0, _p(acts[i]), ci,
                                     _p(nxt), ci, 0, _s()), "mpv_lb_conv(backward-data)")
            dz, dzs = nxt, ci
        return workspace

    def adam(self, lr=2e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        _L.check(_L.lib().mpv_lb_adam(_p(self.params), _p(self.m), _p(self.v), _p(self.grad), self.size,
                                      lr, b1, b2, eps, self.step, _s()), "mpv_lb_adam")
        self.pack()

    # ---- checkpoints (numpy .npz, no pickled objects)
    def state(self, extra: dict | None = None, weights_only: bool = False) -> dict:
        torch.cuda.synchronize()
        st = {"params": self.params.cpu().numpy(), "step": np.array([self.step], np.int64)}
        if not weights_only:
            st["m"], st["v"] = self.m.cpu().numpy(), self.v.cpu().numpy()
        if extra:
            st["extra"] = np.frombuffer(json.dumps(extra).encode(), dtype=np.uint8)
        return st

    def save(self, path: str, extra: dict | None = None, weights_only: bool = False):
        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        buf = io.BytesIO()
        np.savez(buf, **self.state(extra, weights_only))
        tmp = path + ".tmp"
        with open(tmp, "wb") as f:
            f.write(buf.getvalue())
        os.replace(tmp, path)

    @classmethod
    def load(cls, path: str, device="cuda"):
        with np.load(path, allow_pickle=False) as z:
            net = cls(device, params=z["params"])
            net.step = int(z["step"][0])
            if "m" in z:
                net.m.copy_(torch.from_numpy(z["m"]))
                net.v.copy_(torch.from_numpy(z["v"]))
            extra = json.loads(bytes(z["extra"]).decode()) if "extra" in z else {}
        return net, extra


def coarse_images(left, right, levels: int = 3):
    """The coarsest pyramid images (levels-1 halvings) of a pair, computed by mpv_downsample."""
    for _ in range(levels - 1):
        left, right = mpv.downsample(left), mpv.downsample(right)
    return left, right


class Coarse:
    """Coarse-level MPV + features for one coarse shape (workspace held)."""

    def __init__(self, params: mpv.MPVParams, w0: int, h0: int, device="cuda"):
        self.params = params
        p = params.c()
        need = int(_L.lib().mpv_lb_coarse_workspace_bytes(C.byref(p), w0, h0))
        if need == 0:
            raise _L.MPVError(_L.MPV_ERR_INVALID_ARG, "mpv_lb_coarse_workspace_bytes")
        self.ws = torch.empty(need, dtype=torch.uint8, device=device)
        self.w0, self.h0 = w0, h0

    def __call__(self, left0, right0, feat=None, raw=None, disp=None):
        li, ri = mpv._image(left0, "left0"), mpv._image(right0, "right0")
        dev = left0.device
        feat = torch.empty((self.h0, self.w0, 8), dtype=torch.int16, device=dev) if feat is None else feat
        raw = torch.empty((self.h0, self.w0), dtype=torch.int16, device=dev) if raw is None else raw
        disp = torch.empty((self.h0, self.w0), dtype=torch.int16, device=dev) if disp is None else disp
        p = self.params.c()
        _L.check(_L.lib().mpv_lb_coarse(C.byref(p), C.byref(li), C.byref(ri), _p(feat), _p(raw), _p(disp),
                                        _p(self.ws), self.ws.numel(), _s()), "mpv_lb_coarse")
        return feat, raw, disp


def loss(o, raw0, labels, beta, inv_count, dz=None, partials=None):
    n, hc, wc, _ = o.shape
    H, W = labels.shape[-2:]
    dz = torch.empty((n, hc, wc, 4), dtype=torch.int16, device=o.device) if dz is None else dz
    nb = (n * hc * wc + 255) // 256
    partials = torch.empty(nb, dtype=torch.float32, device=o.device) if partials is None else partials
    _L.check(_L.lib().mpv_lb_loss(_p(o), _p(raw0), _p(labels), n, hc, wc, H, W, beta, inv_count, _p(dz),
                                  _p(partials), _s()), "mpv_lb_loss")
    return dz, partials


def bands(o, raw0, W, H, D, theta, lo=None, ln=None, nlow=None):
    """Fine-level bands of one image from the network output o [hc][wc][4]."""
    hc, wc, _ = o.shape
    dev = o.device
    lo = torch.empty((H, W), dtype=torch.int16, device=dev) if lo is None else lo
    ln = torch.empty((H, W), dtype=torch.uint8, device=dev) if ln is None else ln
    nlow = torch.empty(1, dtype=torch.int32, device=dev) if nlow is None else nlow
    _L.check(_L.lib().mpv_lb_bands(_p(o), _p(raw0), wc, hc, W, H, D, theta, _p(lo), _p(ln), _p(nlow), _s()),
             "mpv_lb_bands")
    return lo, ln, nlow


@dataclass
class LearnedConfig:
    levels: int = 3          # the network reads the coarsest of this many levels
    theta: float = 0.5       # confidence threshold of a coarse pixel
    fallback_frac: float = 0.05  # frames with more low-confidence coarse pixels run full range
    cap: int = 16            # widest band


class LearnedMatcher:
    """Learned-band MPV for one frame shape: coarse level -> network -> fine bands ->
    banded finest level (mpv_match), or plain full-range MPV for a fallback frame."""

    def __init__(self, net: BandNet, params: mpv.MPVParams, width: int, height: int,
                 cfg: LearnedConfig | None = None, device="cuda"):
        self.net, self.params, self.cfg = net, params, cfg or LearnedConfig()
        self.W, self.H = width, height
        s = self.cfg.levels - 1
        self.w0, self.h0 = width >> s, height >> s
        d0 = -(-params.num_disp // (1 << s))
        self.coarse = Coarse(mpv.MPVParams(num_disp=d0, num_paths=params.num_paths, lam=params.lam,
                                           tau=params.tau, lr_max_diff=params.lr_max_diff), self.w0, self.h0, device)
        self.lo = torch.empty((height, width), dtype=torch.int16, device=device)
        self.len = torch.empty((height, width), dtype=torch.uint8, device=device)
        self.nlow = torch.zeros(1, dtype=torch.int32, device=device)
        self.nlow_host = torch.zeros(1, dtype=torch.int32).pin_memory()
        band = mpv.Band(self.lo, self.cfg.cap, self.len)
        self.band = band
        self.ws = torch.empty(max(mpv.match_workspace_bytes(params, width, height, band),
                                  mpv.match_workspace_bytes(params, width, height)), dtype=torch.uint8,
                              device=device)
        self.disp = torch.empty((height, width), dtype=torch.int16, device=device)
        self.proposed = torch.cuda.Event()
        self.fallbacks = 0
        self.frames = 0
        self.last_fallback = False

    def propose(self, left, right):
        """Enqueue the coarse level, the network and the fine bands on the current stream;
        the low-confidence count is copied into pinned host memory behind the `proposed`
        event (nothing waits here)."""
        l0, r0 = coarse_images(left, right, self.cfg.levels)
        feat, raw0, _ = self.coarse(l0, r0)
        o, _ = self.net.forward(feat.unsqueeze(0))
        bands(o[0], raw0, self.W, self.H, self.params.num_disp, self.cfg.theta, self.lo, self.len, self.nlow)
        self.nlow_host.copy_(self.nlow, non_blocking=True)
        self.proposed.record()
        return o

    def ready(self) -> bool:
        """True once the last proposal's low-confidence count has reached the host."""
        return self.proposed.query()

    def fallback_due(self) -> bool:
        """Whether the last proposal sends its frame to full-range matching (call once ready)."""
        return int(self.nlow_host[0]) > self.cfg.fallback_frac * self.w0 * self.h0

    def finish(self, left, right, fallback: bool):
        """Enqueue the finest level: the proposed bands, or plain full range for a fallback."""
        self.frames += 1
        self.last_fallback = fallback
        self.fallbacks += int(fallback)
        return mpv.match(left, right, self.params, None if fallback else self.band, workspace=self.ws)

    def __call__(self, left, right, allow_fallback=True):
        """Disparity of one frame. With the fallback on, the call waits for this frame's
        proposal event (the count decides which finest level to enqueue); a pipeline that
        keeps several frames in flight calls propose / ready / finish instead and never
        waits (serve.LearnedGpuExecutor)."""
        self.propose(left, right)
        fb = False
        if allow_fallback:
            self.proposed.synchronize()
            fb = self.fallback_due()
        return self.finish(left, right, fb)


# ---------------------------------------------------------------------------------------
# Training data and loop
# ---------------------------------------------------------------------------------------
def scene_specs(first_seed: int, count: int, width=1280, height=720, num_disp=128):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([first_seed, count])))
    planes = rng.integers(20, 41, count)
    return [(first_seed + i, width, height, num_disp, int(k)) for i, k in enumerate(planes)]


class Dataset:
    """Features, coarse winners and plain-MPV labels of a list of scenes, resident on the GPU.
    Scenes are generated on the host in chunks (worker processes) and dropped once labelled."""

    def __init__(self, specs, params: mpv.MPVParams, levels=3, device="cuda", workers=16, chunk=64,
                 log=None):
        from .scene import scene_chunks
        _, W, H, D, _ = specs[0]
        s = levels - 1
        self.W, self.H, self.hc, self.wc = W, H, H >> s, W >> s
        n = len(specs)
        d0 = -(-D // (1 << s))
        cparams = mpv.MPVParams(num_disp=d0, num_paths=params.num_paths, lam=params.lam, tau=params.tau,
                                lr_max_diff=params.lr_max_diff)
        coarse = Coarse(cparams, self.wc, self.hc, device)
        plain = mpv.Pyramid(params, W, H, levels=1, radius=4, device=device)
        self.feat = torch.empty((n, self.hc, self.wc, 8), dtype=torch.int16, device=device)
        self.raw0 = torch.empty((n, self.hc, self.wc), dtype=torch.int16, device=device)
        self.labels = torch.empty((n, H, W), dtype=torch.int16, device=device)
        disp0 = torch.empty((self.hc, self.wc), dtype=torch.int16, device=device)
        i = 0
        for scenes in scene_chunks(specs, workers=workers, chunk=chunk):
            for sc in scenes:
                L = torch.from_numpy(sc.left).to(device)
                R = torch.from_numpy(sc.right).to(device)
                l0, r0 = coarse_images(L, R, levels)
                coarse(l0, r0, self.feat[i], self.raw0[i], disp0)
                self.labels[i].copy_(plain(L, R))
                i += 1
            if log:
                log(f"dataset: {i}/{n} pairs labelled")
        torch.cuda.synchronize()
        covered = self.labels[:, : 4 * self.hc, : 4 * self.wc] >= 0
        self.counts = covered.reshape(n, -1).sum(dim=1).cpu().numpy().astype(np.int64)
        self.n = n


def dataset_loss(net: BandNet, data: Dataset, beta: float = 0.05, batch: int = 8) -> float:
    """Mean loss over every labelled pixel of the dataset (forward only, fixed order)."""
    total = 0.0
    count = int(data.counts.sum())
    for i in range(0, data.n, batch):
        j = min(i + batch, data.n)
        o, _ = net.forward(data.feat[i:j])
        _, parts = loss(o, data.raw0[i:j], data.labels[i:j], beta, 1.0 / max(count, 1))
        total += float(parts.double().sum().item())
    return total


def train(net: BandNet, data: Dataset, steps: int, batch: int = 8, lr: float = 2e-3, beta: float = 0.05,
          seed: int = 0, start_step: int = 0, rng_state: dict | None = None, ckpt: str | None = None,
          ckpt_every: int = 0, log_every: int = 50, log=print):
    """Adam on the masters; batches drawn by a seeded generator (state saved in checkpoints)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    if rng_state is not None:
        rng.bit_generator.state = rng_state
    history = []
    ws = None
    for step in range(start_step, steps):
        idx = rng.integers(0, data.n, batch)
        feat = data.feat[idx]
        raw0 = data.raw0[idx]
        labels = data.labels[idx]
        count = int(data.counts[idx].sum())
        o, acts = net.forward(feat)
        dz, parts = loss(o, raw0, labels, beta, 1.0 / max(count, 1))
        ws = net.backward(acts, dz, ws)
        net.adam(lr=lr)
        if log_every and (step + 1) % log_every == 0:
            lval = float(parts.sum().item())
            history.append((step + 1, lval))
            log(f"step {step + 1}: loss {lval:.4f}")
        if ckpt and ckpt_every and (step + 1) % ckpt_every == 0:
            net.save(ckpt, {"step": step + 1, "rng": rng.bit_generator.state, "seed": seed})
    return history, rng.bit_generator.state


# ---------------------------------------------------------------------------------------
# Evaluation: learned bands vs the fixed +-radius pyramid vs plain full-range MPV
# ---------------------------------------------------------------------------------------
def compare_to_plain(disp, plain):
    """Plain-valid pixels where `disp` is invalid, and where it is valid but more than 1 away."""
    valid = plain >= 0
    inv = valid & (disp < 0)
    dif = valid & (disp >= 0) & ((disp.int() - plain.int()).abs() > 1)
    return int(inv.sum()), int(dif.sum()), int(valid.sum())


def gt_errors(disp, gt, occluded):
    """Non-occluded pixels whose disparity is invalid or more than 1 from the ground truth."""
    m = ~occluded
    err = m & ((disp < 0) | ((disp.int() - gt.int()).abs() > 1))
    return int(err.sum()), int(m.sum())


def evaluate(net: BandNet, specs, params: mpv.MPVParams, cfg: LearnedConfig | None = None, workers=16,
             radius=4, log=None):
    """Bad-pixel rates against plain MPV (split into invalid / off by more than 1) and error
    rates against the ground truth, for plain, the fixed-band pyramid, and learned bands with
    and without the per-frame fallback."""
    from .scene import scene_chunks
    cfg = cfg or LearnedConfig()
    _, W, H, _, _ = specs[0]
    plain = mpv.Pyramid(params, W, H, levels=1)
    fixed = mpv.Pyramid(params, W, H, levels=cfg.levels, radius=radius)
    lm = LearnedMatcher(net, params, W, H, cfg)
    names = ["plain", f"fixed_pm{radius}", "learned_banded", "learned"]
    acc = {k: dict(inv=0, dif=0, valid=0, max_pair=0.0, gt_err=0, gt_n=0) for k in names}
    frames = 0
    for scenes in scene_chunks(specs, workers=workers, chunk=32):
        for sc in scenes:
            L = torch.from_numpy(sc.left).cuda()
            R = torch.from_numpy(sc.right).cuda()
            gt = torch.from_numpy(sc.disp).cuda()
            occ = torch.from_numpy(sc.occluded).cuda()
            ref = plain(L, R).clone()
            banded = lm(L, R, allow_fallback=False).clone()
            lm.proposed.synchronize()
            fb = lm.fallback_due()
            lm.fallbacks += int(fb)
            outs = {"plain": ref, names[1]: fixed(L, R), "learned_banded": banded,
                    "learned": ref if fb else banded}
            for k, d in outs.items():
                i, df, n = compare_to_plain(d, ref)
                e, g = gt_errors(d, gt, occ)
                a = acc[k]
                a["inv"] += i
                a["dif"] += df
                a["valid"] += n
                a["max_pair"] = max(a["max_pair"], (i + df) / max(n, 1))
                a["gt_err"] += e
                a["gt_n"] += g
            frames += 1
        if log:
            log(f"evaluate: {frames}/{len(specs)} pairs")
    res = {}
    for k, a in acc.items():
        res[k] = {"bad_vs_plain": (a["inv"] + a["dif"]) / max(a["valid"], 1),
                  "invalid_vs_plain": a["inv"] / max(a["valid"], 1),
                  "differ_vs_plain": a["dif"] / max(a["valid"], 1),
                  "max_pair_bad_vs_plain": a["max_pair"],
                  "err_gt": a["gt_err"] / max(a["gt_n"], 1)}
    res["fallback_frac"] = lm.fallbacks / max(frames, 1)
    res["pairs"] = frames
    return res


def _main(argv=None):
    import argparse
    import time
    ap = argparse.ArgumentParser(description="Train the band-proposal network on seeded synthetic pairs "
                                             "labelled by plain full-range MPV, then evaluate held-out pairs.")
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--first-seed", type=int, default=40000)
    ap.add_argument("--eval-pairs", type=int, default=200)
    ap.add_argument("--eval-seed", type=int, default=42000)
    ap.add_argument("--width", type=int, default=1280)
    ap.add_argument("--height", type=int, default=720)
    ap.add_argument("--num-disp", type=int, default=128)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--beta", type=float, default=0.05)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--ckpt", default=None)
    ap.add_argument("--resume", action="store_true")
    ap.add_argument("--workers", type=int, default=16)
    a = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)  # noqa: E731
    params = mpv.MPVParams(num_disp=a.num_disp, num_paths=8)
    t0 = time.time()
    specs = scene_specs(a.first_seed, a.pairs, a.width, a.height, a.num_disp)
    data = Dataset(specs, params, workers=a.workers, log=log)
    log(f"dataset ready in {time.time() - t0:.1f} s")
    start, rng_state = 0, None
    if a.resume and a.ckpt and os.path.exists(a.ckpt):
        net, extra = BandNet.load(a.ckpt)
        start, rng_state = extra["step"], extra["rng"]
    else:
        net = BandNet("cuda", seed=a.seed)
    t1 = time.time()
    hist, _ = train(net, data, a.steps, batch=a.batch, lr=a.lr, beta=a.beta, seed=a.seed, start_step=start,
                    rng_state=rng_state, ckpt=a.ckpt, ckpt_every=500 if a.ckpt else 0, log_every=100, log=log)
    torch.cuda.synchronize()
    log(f"trained {a.steps - start} steps in {time.time() - t1:.1f} s")
    meta = {"pairs": a.pairs, "first_seed": a.first_seed, "steps": a.steps, "batch": a.batch, "lr": a.lr,
            "beta": a.beta, "seed": a.seed, "shape": [a.width, a.height, a.num_disp],
            "loss_history": hist}
    if a.eval_pairs:
        del data
        res = evaluate(net, scene_specs(a.eval_seed, a.eval_pairs, a.width, a.height, a.num_disp), params,
                       workers=a.workers, log=log)
        meta["eval"] = res
        log(json.dumps(res, indent=1))
    net.save(a.out, meta, weights_only=True)
    log(f"saved {a.out}")


if __name__ == "__main__":
    _main()
