"""CPU oracle for the multi-scale MPV stereo matcher — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this package.
The product library never imports, links or executes anything here, and this package
imports nothing from the product (it takes numpy arrays and returns numpy arrays).

The arithmetic lives in ``mpv_oracle.c`` (plain C, int64, OpenMP over independent
lines); this file builds it with gcc, binds it with ctypes and composes the steps of the
multi-scale pipeline (Section 3.4) in the paper's order: pyramid, per-level cost,
per-path Viterbi energies (Section 3.2, eq. e(p,u); Section 3.3 fast technique), their
sum or the paper's layered merge (Section 3.2, Table alg), winner-take-all, left-right
check, then the band for the next level.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mpv_oracle.c")
LIB = os.path.join(HERE, "libmpv_oracle.so")

DEFINITION = 0
FAST = 1
INF = np.iinfo(np.int64).max // 4

# scan directions r = (dx, dy): L->R, R->L, T->B, B->T, TL->BR, BR->TL, TR->BL, BL->TR
DIRECTIONS = [(+1, 0), (-1, 0), (0, +1), (0, -1), (+1, +1), (-1, -1), (-1, +1), (+1, -1)]


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        lib = C.CDLL(LIB)
        P = C.c_void_p
        i32 = C.c_int
        lib.orc_downsample.argtypes = [P, i32, i32, P]
        lib.orc_census5x5.argtypes = [P, i32, i32, P]
        lib.orc_cost.argtypes = [P, P, i32, i32, P, P, i32, P]
        lib.orc_path.argtypes = [P, i32, i32, i32, P, P, i32, i32, i32, i32, i32, P]
        lib.orc_path.restype = i32
        lib.orc_aggregate.argtypes = [P, i32, i32, i32, P, P, i32, i32, C.c_uint32, i32, i32, i32,
                                      P, P, P]
        lib.orc_aggregate.restype = i32
        lib.orc_layered.argtypes = [P, i32, i32, i32, P, P, i32, i32, i32, i32, i32, i32, P, P]
        lib.orc_layered.restype = i32
        lib.orc_path_g.argtypes = [P, i32, i32, i32, P, P, i32, i32, i32, i32, P, i32, i32, P]
        lib.orc_path_g.restype = i32
        lib.orc_aggregate_g.argtypes = [P, i32, i32, i32, P, P, i32, i32, C.c_uint32, i32, i32, P, i32,
                                        i32, P, P, P]
        lib.orc_aggregate_g.restype = i32
        lib.orc_layered_g.argtypes = [P, i32, i32, i32, P, P, i32, i32, i32, i32, i32, P, i32, i32, P, P]
        lib.orc_layered_g.restype = i32
        lib.orc_grad_weight.argtypes = [i32, i32, i32]
        lib.orc_grad_weight.restype = i32
        lib.orc_set_threads.argtypes = [i32]
        lib.orc_set_threads.restype = i32
        lib.orc_wta_lr.argtypes = [P, i32, i32, i32, P, P, i32, i32, P, P, P]
        lib.orc_propagate.argtypes = [P, i32, i32, i32, i32, i32, i32, P]
        lib.orc_propagate.restype = i32
        lib.orc_propagate_block.argtypes = [P, i32, i32, i32, i32, i32, i32, i32, P]
        lib.orc_propagate_block.restype = i32
        lib.orc_propagate_interp.argtypes = [P, i32, i32, i32, i32, i32, i32, P]
        lib.orc_propagate_interp.restype = i32
        lib.orc_ssim_patch_cost.argtypes = [P, P]
        lib.orc_ssim_patch_cost.restype = i32
        lib.orc_ssim_ratio_parts.argtypes = [P, P, P, P, P, P]
        lib.orc_ssim_cost.argtypes = [P, P, i32, i32, P, P, i32, P]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def downsample(img: np.ndarray) -> np.ndarray:
    img = _c(img, np.uint8)
    h, w = img.shape
    out = np.empty((h // 2, w // 2), np.uint8)
    _load().orc_downsample(_p(img), w, h, _p(out))
    return out


def census(img: np.ndarray) -> np.ndarray:
    img = _c(img, np.uint8)
    h, w = img.shape
    out = np.empty((h, w), np.uint32)
    _load().orc_census5x5(_p(img), w, h, _p(out))
    return out


def cost(cl, cr, num_disp, lo=None, length=None, cap=None) -> np.ndarray:
    cl, cr = _c(cl, np.uint32), _c(cr, np.uint32)
    h, w = cl.shape
    cap = num_disp if cap is None else cap
    lo, length = _c(lo, np.int16), _c(length, np.uint8)
    out = np.empty((h, w, cap), np.uint8)
    _load().orc_cost(_p(cl), _p(cr), w, h, _p(lo), _p(length), cap, _p(out))
    return out


def ssim_patch_cost(psi, phi) -> int:
    """Quantised SSIM cost (eq. ssim, 0 .. 24) of two 5x5 uint8 patches."""
    psi, phi = _c(psi, np.uint8).reshape(25), _c(phi, np.uint8).reshape(25)
    return int(_load().orc_ssim_patch_cost(_p(psi), _p(phi)))


def ssim_ratio(psi, phi) -> tuple[int, int]:
    """The SSIM index of two 5x5 patches as the exact ratio (num, den), den > 0."""
    psi, phi = _c(psi, np.uint8).reshape(25), _c(phi, np.uint8).reshape(25)
    parts = [np.zeros(1, np.int64), np.zeros(1, np.uint64), np.zeros(1, np.int64), np.zeros(1, np.uint64)]
    _load().orc_ssim_ratio_parts(_p(psi), _p(phi), *[_p(a) for a in parts])
    num = (int(parts[0][0]) << 64) | int(parts[1][0])
    den = (int(parts[2][0]) << 64) | int(parts[3][0])
    return num, den


def ssim_cost(left, right, num_disp, lo=None, length=None, cap=None) -> np.ndarray:
    """SSIM cost volume [H][W][cap] (slot j = disparity lo + j, 24 where x - d < 0, 0xFF
    past a pixel's band): the SSIM data term of Section 3.2 in place of the census cost."""
    left, right = _c(left, np.uint8), _c(right, np.uint8)
    h, w = left.shape
    cap = num_disp if cap is None else cap
    lo, length = _c(lo, np.int16), _c(length, np.uint8)
    out = np.empty((h, w, cap), np.uint8)
    _load().orc_ssim_cost(_p(left), _p(right), w, h, _p(lo), _p(length), cap, _p(out))
    return out


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops; returns the previous maximum."""
    return int(_load().orc_set_threads(n))


def grad_weight(lam, sigma, g):
    """Gradient-weighted TV weight of eq. EU for an intensity difference g."""
    return int(_load().orc_grad_weight(lam, sigma, g))


def path(cost_vol, num_disp, r, lam, tau, lo=None, length=None, mode=FAST, img=None, sigma=0) -> np.ndarray:
    """Energies of direction r; img (left image) and sigma > 0: gradient-weighted TV."""
    cost_vol = _c(cost_vol, np.uint8)
    h, w, cap = cost_vol.shape
    lo, length, img = _c(lo, np.int16), _c(length, np.uint8), _c(img, np.uint8)
    out = np.empty((h, w, cap), np.int64)
    rc = _load().orc_path_g(_p(cost_vol), w, h, num_disp, _p(lo), _p(length), cap, r, lam, tau, _p(img),
                            sigma, mode, _p(out))
    assert rc == 0
    return out


def aggregate(cost_vol, num_disp, num_paths, lam, tau, lo=None, length=None, path_mask=0,
              mode=FAST, per_path=False, img=None, sigma=0):
    cost_vol = _c(cost_vol, np.uint8)
    h, w, cap = cost_vol.shape
    lo, length, img = _c(lo, np.int16), _c(length, np.uint8), _c(img, np.uint8)
    S = np.empty((h, w, cap), np.int64)
    scratch = np.empty((h, w, cap), np.int64)
    pp = np.zeros((8, h, w, cap), np.int64) if per_path else None
    rc = _load().orc_aggregate_g(_p(cost_vol), w, h, num_disp, _p(lo), _p(length), cap, num_paths,
                                 path_mask, lam, tau, _p(img), sigma, mode, _p(S), _p(scratch), _p(pp))
    assert rc == 0
    return (S, pp) if per_path else S


def layered(cost_vol, num_disp, num_layers, lam, tau, lo=None, length=None, occ=False, mode=FAST,
            per_layer=False, img=None, sigma=0):
    """The paper's hierarchical merge (Section 3.2, Table alg): layer k merges directions
    2k and 2k+1 over the previous layer's merged energy (the cost for k = 0); min for the
    horizontal layer, floor mean for the others. Returns M [H][W][cap] (int64, absent
    slots INF), and every layer's merged energies when per_layer."""
    cost_vol = _c(cost_vol, np.uint8)
    h, w, cap = cost_vol.shape
    lo, length, img = _c(lo, np.int16), _c(length, np.uint8), _c(img, np.uint8)
    M = np.empty((h, w, cap), np.int64)
    pl = np.zeros((num_layers, h, w, cap), np.int64) if per_layer else None
    rc = _load().orc_layered_g(_p(cost_vol), w, h, num_disp, _p(lo), _p(length), cap, num_layers, lam,
                               tau, 1 if occ else 0, _p(img), sigma, mode, _p(M), _p(pl))
    assert rc == 0
    return (M, pl) if per_layer else M


def wta_lr(S, num_disp, lr_max_diff, lo=None, length=None):
    S = _c(S, np.int64)
    h, w, cap = S.shape
    lo, length = _c(lo, np.int16), _c(length, np.uint8)
    dl = np.empty((h, w), np.int16)
    dr = np.empty((h, w), np.int16)
    out = np.empty((h, w), np.int16)
    _load().orc_wta_lr(_p(S), w, h, num_disp, _p(lo), _p(length), cap, lr_max_diff, _p(dl),
                       _p(dr), _p(out))
    return dl, dr, out


def propagate(dl_coarse, width, height, level_disp, radius):
    dl_coarse = _c(dl_coarse, np.int16)
    hc, wc = dl_coarse.shape
    lo = np.empty((height, width), np.int16)
    cap = _load().orc_propagate(_p(dl_coarse), wc, hc, width, height, level_disp, radius, _p(lo))
    return lo, cap


def propagate_block(dl_coarse, width, height, level_disp, radius, block):
    """Section 3.4, intermediate layer: each block of block x block pixels searches around
    twice the mode of its parents' raw disparities."""
    dl_coarse = _c(dl_coarse, np.int16)
    hc, wc = dl_coarse.shape
    lo = np.empty((height, width), np.int16)
    cap = _load().orc_propagate_block(_p(dl_coarse), wc, hc, width, height, level_disp, radius, block, _p(lo))
    return lo, cap


def propagate_interp(dl_coarse, width, height, level_disp, radius):
    """Section 3.4, last layer: sampled pixels take twice the coarse raw disparity, the
    others the linear interpolation of the samples around them."""
    dl_coarse = _c(dl_coarse, np.int16)
    hc, wc = dl_coarse.shape
    lo = np.empty((height, width), np.int16)
    cap = _load().orc_propagate_interp(_p(dl_coarse), wc, hc, width, height, level_disp, radius, _p(lo))
    return lo, cap


def level_block(levels: int, level: int, block: int) -> int:
    """Block side of intermediate layer `level` (1 .. levels-2) of the paper's propagation:
    `block` at layer 1, halved at every finer layer (never below 2); the last layer uses
    single-pixel blocks with interpolation (Section 3.4)."""
    return max(block >> (level - 1), 2)


def level_disparities(num_disp: int, levels: int) -> list[int]:
    """D_l = ceil(D / 2^(L-1-l)): the top layer searches a quarter of the range for L=3
    (Section 3.4)."""
    return [-(-num_disp // (1 << (levels - 1 - l))) for l in range(levels)]


@dataclass
class LevelResult:
    width: int
    height: int
    num_disp: int
    cap: int
    lo: np.ndarray | None
    dl: np.ndarray
    dr: np.ndarray
    out: np.ndarray
    S: np.ndarray | None = field(default=None, repr=False)


def pyramid(left, right, num_disp, levels=3, radius=4, num_paths=8, lam=8, tau=4,
            lr_max_diff=1, mode=FAST, keep_sums=False, bands=None, merge="sum", occ=False,
            grad_sigma=0, propagation="nearest", block=8, data_term="census"):
    """Multi-scale MPV (Section 3.4). Level 0 is the coarsest and searches its full range;
    every finer level searches the band propagated from the level above. ``levels=1`` is
    plain single-scale MPV. ``bands`` optionally replaces the finest level's band by a
    given (lo, len, cap) triple (the learned-band path). ``merge`` = "sum" sums the
    ``num_paths`` directed paths; "layered" runs num_paths / 2 layers of the paper's
    hierarchical merge (``occ``: its occlusion strategy) and takes decisions on the last
    layer's merged energies. ``grad_sigma`` > 0 weights every transition by the left image's
    gradient along the path (eq. EU), on each level's own left image. ``propagation`` =
    "nearest" centres every finer pixel's band on twice its parent's raw disparity;
    "paper" is Section 3.4's scheme: block modes (``block`` pixels at layer 1, see
    level_block) at intermediate layers and linear interpolation at the last layer.
    ``data_term`` = "census" (Hamming cost of 5x5 census signatures) or "ssim" (the SSIM cost
    of Section 3.2 on each level's own images)."""
    assert merge in ("sum", "layered")
    assert data_term in ("census", "ssim")
    assert propagation in ("nearest", "paper")
    imgs = [_c(left, np.uint8)], [_c(right, np.uint8)]
    for _ in range(levels - 1):
        imgs[0].insert(0, downsample(imgs[0][0]))
        imgs[1].insert(0, downsample(imgs[1][0]))
    dls = level_disparities(num_disp, levels)
    results = []
    for l in range(levels):
        L_img, R_img = imgs[0][l], imgs[1][l]
        h, w = L_img.shape
        Dl = dls[l]
        length = None
        if l == 0:
            lo, cap = None, Dl
        else:
            prev = results[-1]
            if propagation == "nearest":
                lo, cap = propagate(prev.dl, w, h, Dl, radius)
            elif l == levels - 1:
                lo, cap = propagate_interp(prev.dl, w, h, Dl, radius)
            else:
                lo, cap = propagate_block(prev.dl, w, h, Dl, radius, level_block(levels, l, block))
        if bands is not None and l == levels - 1:
            lo, length, cap = bands
        if data_term == "census":
            cv = cost(census(L_img), census(R_img), Dl, lo, length, cap)
        else:
            cv = ssim_cost(L_img, R_img, Dl, lo, length, cap)
        g = L_img if grad_sigma > 0 else None
        if merge == "sum":
            S = aggregate(cv, Dl, num_paths, lam, tau, lo, length, mode=mode, img=g, sigma=grad_sigma)
        else:
            S = layered(cv, Dl, num_paths // 2, lam, tau, lo, length, occ=occ, mode=mode, img=g,
                        sigma=grad_sigma)
        dl, dr, out = wta_lr(S, Dl, lr_max_diff, lo, length)
        results.append(LevelResult(w, h, Dl, cap, lo, dl, dr, out, S if keep_sums else None))
    return results
