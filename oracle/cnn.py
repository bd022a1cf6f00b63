"""CPU reference of the learned band-proposal network — TEST INFRASTRUCTURE ONLY.

Plain numpy in float64, written from the definitions below; the HIP kernels are checked
against it layer by layer. Not part of the paper: the network proposes, per coarse pixel,
a disparity band for the finest level so that level searches only that band (the paper's
per-pixel search scopes of Section 3.4, here predicted instead of propagated).

Features (8 channels) of a coarse (level-0) pixel p, from the sum of path energies S of
that level (eq. viterbi) with S'(p,d) = S(p,d) - min_d S(p,d), raw winner dl, LR result:
  0: I(p)/255        1: dl/D0            2: [LR-valid]
  3: S'(dl-1)/Z      4: S'(dl+1)/Z       5: S'(dl-2)/Z      6: S'(dl+2)/Z
     (disparities clamped to [0, D0-1]; Z = P * (24 + lambda*min(tau, D0-1)))
  7: min over |d-dl| > 1 of S'(d) / Z   (1 if no such d)
Network: five 3x3 convolutions, zero padding, stride 1, channels 8 -> 32 -> 32 -> 32 ->
32 -> 3, ReLU after the first four. Arrays are NHWC: x[n, y, x, c]; weights w[ky, kx, cin,
cout] (tap (ky, kx) reads input pixel (y + ky - 1, x + kx - 1)).
Heads of output o = (o0, o1, o2) at coarse pixel p (fine disparity units, 4x the coarse):
  center = 4*dl + o0,  width = 2 + clamp(o1, 0, 14),  conf = clamp(o2, 0, 1).
Loss over the fine pixels q of the 4x4 block of p that have a label d* (plain MPV, LR-valid):
  smoothL1(center - d*) + max(0, 2|d* - center| + 2 - width) + beta*width
  + (conf - [|d* - center| <= width/2])^2,
averaged over all labelled fine pixels of the batch; the indicator is a constant.
"""
from __future__ import annotations

import numpy as np


CHANNELS = [8, 32, 32, 32, 32, 3]


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float64/float32 values to bfloat16 (round to nearest, ties to even) and return
    them as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def features(img0, dl, out, S, num_paths, lam, tau):
    """img0 uint8 [H][W]; dl, out int16 [H][W]; S int64 [H][W][D0] (full range)."""
    H, W, D0 = S.shape
    Z = float(num_paths * (24 + lam * max(1, min(tau, D0 - 1))))
    Sp = S - S.min(axis=2, keepdims=True)
    f = np.zeros((H, W, 8))
    f[..., 0] = img0 / 255.0
    f[..., 1] = dl / float(D0)
    f[..., 2] = (out >= 0).astype(np.float64)
    yy, xx = np.mgrid[0:H, 0:W]
    for c, off in zip((3, 4, 5, 6), (-1, +1, -2, +2)):
        d = np.clip(dl.astype(np.int64) + off, 0, D0 - 1)
        f[..., c] = Sp[yy, xx, d] / Z
    far = np.abs(np.arange(D0)[None, None, :] - dl[..., None].astype(np.int64)) > 1
    masked = np.where(far, Sp, np.iinfo(np.int64).max)
    m = masked.min(axis=2)
    f[..., 7] = np.where(far.any(axis=2), m / Z, 1.0)
    return f


def conv3x3(x, w, b):
    """x [N,H,W,Cin], w [3,3,Cin,Cout], b [Cout] -> [N,H,W,Cout]; zero padding."""
    N, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((N, H, W, w.shape[3])) + b
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("nhwc,cd->nhwd", xp[:, ky:ky + H, kx:kx + W, :], w[ky, kx])
    return y


def conv3x3_backward(x, w, dy):
    """Gradients of conv3x3 wrt x, w, b given dy = dL/dy."""
    N, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dw = np.zeros_like(w)
    dxp = np.zeros_like(xp)
    for ky in range(3):
        for kx in range(3):
            dw[ky, kx] = np.einsum("nhwc,nhwd->cd", xp[:, ky:ky + H, kx:kx + W, :], dy)
            dxp[:, ky:ky + H, kx:kx + W, :] += np.einsum("nhwd,cd->nhwc", dy, w[ky, kx])
    db = dy.sum(axis=(0, 1, 2))
    return dxp[:, 1:H + 1, 1:W + 1, :], dw, db


def forward(x, weights):
    """weights: list of (w, b). Returns the list of layer outputs (post-ReLU except the last)."""
    acts = [x]
    for i, (w, b) in enumerate(weights):
        z = conv3x3(acts[-1], w, b)
        acts.append(np.maximum(z, 0.0) if i + 1 < len(weights) else z)
    return acts


def heads(o, dl):
    center = 4.0 * dl + o[..., 0]
    width = 2.0 + np.clip(o[..., 1], 0.0, 14.0)
    conf = np.clip(o[..., 2], 0.0, 1.0)
    return center, width, conf


def _fine_labels(labels, Hc, Wc):
    """labels int [N,H,W] (fine, -1 = none) -> [N,Hc,Wc,16] block view (-1 padded)."""
    N, H, W = labels.shape
    out = np.full((N, Hc, Wc, 16), -1, dtype=np.int64)
    for by in range(4):
        for bx in range(4):
            ys = np.arange(Hc) * 4 + by
            xs = np.arange(Wc) * 4 + bx
            ok_y, ok_x = ys < H, xs < W
            sub = np.full((N, Hc, Wc), -1, dtype=np.int64)
            sub[:, ok_y[:, None] & ok_x[None, :]] = labels[:, ys[ok_y]][:, :, xs[ok_x]].reshape(N, -1)
            out[..., by * 4 + bx] = sub
    return out


def loss_and_grad(o, dl, labels, beta):
    """o [N,Hc,Wc,3] network output, dl [N,Hc,Wc] coarse raw winner, labels [N,H,W] fine
    plain-MPV disparities (-1 = unlabelled). Returns (loss, dL/do, count)."""
    N, Hc, Wc, _ = o.shape
    lab = _fine_labels(labels, Hc, Wc).astype(np.float64)
    valid = lab >= 0
    center, width, conf = heads(o, dl)
    c = center[..., None]
    w = width[..., None]
    e = c - lab
    sl1 = np.where(np.abs(e) < 1, 0.5 * e * e, np.abs(e) - 0.5)
    h = 2 * np.abs(e) + 2 - w
    hinge = np.maximum(h, 0.0)
    ind = (np.abs(e) <= w / 2).astype(np.float64)
    q = conf[..., None] - ind
    per = sl1 + hinge + beta * w + q * q
    count = int(valid.sum())
    scale = 1.0 / max(count, 1)
    loss = float((per * valid).sum() * scale)
    dsl1 = np.where(np.abs(e) < 1, e, np.sign(e))
    dc = ((dsl1 + np.where(h > 0, 2 * np.sign(e), 0.0)) * valid).sum(axis=-1) * scale
    dw_ = ((beta - (h > 0)) * valid).sum(axis=-1) * scale
    dconf = (2 * q * valid).sum(axis=-1) * scale
    g = np.zeros_like(o)
    g[..., 0] = dc
    g[..., 1] = dw_ * ((o[..., 1] > 0) & (o[..., 1] < 14))
    g[..., 2] = dconf * ((o[..., 2] > 0) & (o[..., 2] < 1))
    return loss, g, count


def backward(acts, weights, g_out):
    """Backward through the network. Returns [(dw, db)] per layer and dL/dx of the input."""
    grads = [None] * len(weights)
    dy = g_out
    for i in range(len(weights) - 1, -1, -1):
        w, _ = weights[i]
        if i + 1 < len(weights):
            dy = dy * (acts[i + 1] > 0)
        dx, dw, db = conv3x3_backward(acts[i], w, dy)
        grads[i] = (dw, db)
        dy = dx
    return grads, dy


def bands(o, dl, W, H, D, theta):
    """Fine-level bands from the heads (inference rounding): center rounded half up, width
    rounded half up then clamped; low confidence widens the band to 16. Returns lo int16
    [H][W], len uint8 [H][W], low-confidence count (coarse pixels)."""
    Hc, Wc = dl.shape
    center, _, conf = heads(o, dl)
    c = np.floor(center + 0.5).astype(np.int64)
    w = 2 + np.clip(np.floor(o[..., 1] + 0.5), 0, 14).astype(np.int64)
    low = conf < theta
    w = np.where(low, 16, w)
    w = np.minimum(w, D)
    lo = np.clip(c - w // 2, 0, D - w)
    fy = np.minimum(np.arange(H) // 4, Hc - 1)
    fx = np.minimum(np.arange(W) // 4, Wc - 1)
    return (lo[fy][:, fx].astype(np.int16), w[fy][:, fx].astype(np.uint8), int(low.sum()))


def init_weights(seed=0):
    """He-normal weights, zero biases (float64)."""
    rng = np.random.default_rng(seed)
    ws = []
    for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
        std = np.sqrt(2.0 / (9 * cin))
        ws.append((rng.normal(0, std, (3, 3, cin, cout)), np.zeros(cout)))
    return ws
