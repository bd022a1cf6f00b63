"""HIP path vs the CPU oracle, element by element, through the C ABI.

Integer work throughout, so every comparison is bit-exact: census, downsampling, cost
volumes, each direction's unnormalised path energies, their sums, WTA / right disparity /
LR-checked maps of the unfused calls, the fused single-level path and the fused pyramid.
Shapes span several lane groups and ragged tails (odd widths and heights, ranges that are
not multiples of the lane layout), bands placed at random, and the degenerate cases of
the method (1-pixel images, D = 1, tau = 1 Potts, tau >= D untruncated, lambda = 0).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2001_09678_amd import mpv as m, _lib
    _lib.lib()  # fails loudly if the HIP library is missing
    return m


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _rand_pair(seed, w, h):
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 256, (h, w), dtype=np.uint8), rng.integers(0, 256, (h, w), dtype=np.uint8))


def _scene_pair(seed, w, h, dmax, planes=6, ground=False):
    from paper_2001_09678_amd.scene import make_scene
    s = make_scene(seed, w, h, dmax, planes, ground=ground)
    return s.left, s.right


def _random_band(rng, w, h, D, cap, varlen):
    lo = rng.integers(0, D - cap + 1, size=(h, w)).astype(np.int16)
    ln = rng.integers(1, cap + 1, size=(h, w)).astype(np.uint8) if varlen else None
    return lo, ln


def _band(m, lo, ln, cap):
    return None if lo is None else m.Band(_cuda(lo), cap, None if ln is None else _cuda(ln))


def _log(*a):
    print(*a, flush=True)


SHAPES = [(1, 1), (7, 1), (1, 9), (33, 17), (70, 45), (129, 66)]


@pytest.mark.parametrize("w,h", SHAPES + [(320, 240)])
def test_census_and_downsample(mpv, orc, w, h):
    _log("census", w, h)
    L, _ = _rand_pair(w * 1000 + h, w, h)
    got = _np(mpv.census(_cuda(L))).view(np.uint32)
    np.testing.assert_array_equal(got, orc.census(L))
    if w >= 2 and h >= 2:
        np.testing.assert_array_equal(_np(mpv.downsample(_cuda(L))), orc.downsample(L))


@pytest.mark.parametrize("w,h,D", [(33, 17, 5), (70, 45, 64), (129, 66, 100), (40, 9, 256), (1, 1, 3)])
def test_cost_full_and_banded(mpv, orc, w, h, D):
    _log("cost", w, h, D)
    L, R = _rand_pair(7 + w, w, h)
    p = mpv.MPVParams(num_disp=D)
    got = _np(mpv.cost(_cuda(L), _cuda(R), p))
    cl, cr = orc.census(L), orc.census(R)
    np.testing.assert_array_equal(got, orc.cost(cl, cr, D))
    rng = np.random.default_rng(w)
    cap = max(1, min(D, 9))
    lo, ln = _random_band(rng, w, h, D, cap, True)
    got = _np(mpv.cost(_cuda(L), _cuda(R), p, _band(mpv, lo, ln, cap)))
    np.testing.assert_array_equal(got, orc.cost(cl, cr, D, lo, ln, cap))


PATH_CASES = [
    # w, h, D, lam, tau, band kind
    (33, 17, 5, 8, 4, None),
    (70, 45, 64, 8, 4, None),
    (129, 66, 100, 8, 4, None),
    (61, 29, 128, 8, 4, None),
    (37, 23, 200, 3, 5, None),
    (45, 31, 32, 8, 1, None),        # Potts
    (45, 31, 20, 5, 40, None),       # tau >= D: untruncated TV
    (40, 20, 17, 0, 4, None),        # lambda = 0
    (1, 1, 7, 8, 4, None),
    (9, 1, 16, 8, 4, None),
    (1, 12, 16, 8, 4, None),
    (70, 45, 64, 8, 4, ("fixed", 9)),
    (70, 45, 128, 8, 4, ("var", 16)),
    (53, 41, 64, 8, 4, ("var", 30)),
    (53, 41, 128, 8, 4, ("var", 60)),   # wider than any lane group: masked full-range scan
    (53, 41, 100, 8, 9, ("var", 20)),
]


@pytest.mark.parametrize("w,h,D,lam,tau,band", PATH_CASES)
def test_path_energies_each_direction(mpv, orc, w, h, D, lam, tau, band):
    _log("paths", w, h, D, lam, tau, band)
    L, R = _rand_pair(w + 31 * h + D, w, h)
    rng = np.random.default_rng(D * 7 + w)
    cl, cr = orc.census(L), orc.census(R)
    if band is None:
        lo = ln = None
        cap = D
    else:
        cap = band[1]
        lo, ln = _random_band(rng, w, h, D, cap, band[0] == "var")
    cv = orc.cost(cl, cr, D, lo, ln, cap)
    p = mpv.MPVParams(num_disp=D, num_paths=8, lam=lam, tau=tau, agg_type="i32")
    cv_t = _cuda(cv)
    b = _band(mpv, lo, ln, cap)
    for r in range(8):
        got = _np(mpv.aggregate(cv_t, p, b, path_mask=1 << r)).astype(np.int64)
        ref = orc.path(cv, D, r, lam, tau, lo, ln)
        inband = ref < orc.INF
        np.testing.assert_array_equal(got[inband], ref[inband], err_msg=f"direction {r}")
        assert (got[~inband] == 0x7FFFFFFF).all()


@pytest.mark.parametrize("P", [1, 2, 4, 8])
@pytest.mark.parametrize("agg", ["u16", "i32"])
def test_sum_and_disparity(mpv, orc, P, agg):
    _log("sum+disparity", P, agg)
    w, h, D = 95, 43, 48
    L, R = _scene_pair(P + 11, w, h, D - 1)
    cl, cr = orc.census(L), orc.census(R)
    cv = orc.cost(cl, cr, D)
    p = mpv.MPVParams(num_disp=D, num_paths=P, agg_type=agg)
    S = _np(mpv.aggregate(_cuda(cv), p))
    S = (S.view(np.uint16) if agg == "u16" else S).astype(np.int64)
    ref = orc.aggregate(cv, D, P, 8, 4)
    np.testing.assert_array_equal(S, ref)
    # WTA / right disparity / LR from the same sums
    dt = np.int16 if agg == "u16" else np.int32
    agg_t = _cuda(ref.astype(np.uint16).view(np.int16) if agg == "u16" else ref.astype(np.int32))
    d, dr, raw = (_np(t) for t in mpv.disparity(agg_t, p))
    rl, rr, ro = orc.wta_lr(ref, D, 1)
    np.testing.assert_array_equal(raw, rl)
    np.testing.assert_array_equal(dr, rr)
    np.testing.assert_array_equal(d, ro)
    assert dt  # silence


def test_disparity_banded_and_lr_off(mpv, orc):
    _log("disparity banded")
    w, h, D, cap = 77, 31, 64, 12
    rng = np.random.default_rng(5)
    lo, ln = _random_band(rng, w, h, D, cap, True)
    S = rng.integers(0, 300, size=(h, w, cap)).astype(np.int64)
    S[np.arange(cap)[None, None, :] >= ln[:, :, None]] = 0x7FFFFFFF
    for lr in (1, 0, 3, -1):
        p = mpv.MPVParams(num_disp=D, lr_max_diff=lr, agg_type="i32")
        d, dr, raw = (_np(t) for t in mpv.disparity(_cuda(S.astype(np.int32)), p, _band(mpv, lo, ln, cap)))
        rl, rr, ro = orc.wta_lr(np.where(S == 0x7FFFFFFF, orc.INF, S), D, lr, lo, ln)
        np.testing.assert_array_equal(raw, rl)
        np.testing.assert_array_equal(dr, rr)
        np.testing.assert_array_equal(d, ro)


MATCH_CASES = [
    (33, 17, 5, 4), (70, 45, 64, 4), (129, 66, 100, 8), (61, 29, 128, 8), (37, 23, 200, 2),
    (40, 20, 32, 1), (1, 1, 4, 8), (5, 70, 16, 8),
]


@pytest.mark.parametrize("w,h,D,P", MATCH_CASES)
def test_fused_match_full_range(mpv, orc, w, h, D, P):
    _log("match", w, h, D, P)
    L, R = _scene_pair(w * 3 + D, w, h, max(D - 1, 0))
    p = mpv.MPVParams(num_disp=D, num_paths=P)
    d, dr, raw = (_np(t) for t in mpv.match(_cuda(L), _cuda(R), p, want_all=True))
    ref = orc.pyramid(L, R, D, levels=1, num_paths=P)[0]
    np.testing.assert_array_equal(raw, ref.dl)
    np.testing.assert_array_equal(dr, ref.dr)
    np.testing.assert_array_equal(d, ref.out)


@pytest.mark.parametrize("cap,varlen,tau", [(9, False, 4), (16, True, 4), (40, True, 4), (5, True, 1), (12, False, 9)])
def test_fused_match_banded(mpv, orc, cap, varlen, tau):
    _log("match banded", cap, varlen, tau)
    w, h, D = 91, 47, 96
    L, R = _scene_pair(cap + 100, w, h, D - 1)
    lo, ln = _random_band(np.random.default_rng(cap), w, h, D, cap, varlen)
    p = mpv.MPVParams(num_disp=D, num_paths=8, tau=tau)
    d, dr, raw = (_np(t) for t in mpv.match(_cuda(L), _cuda(R), p, _band(mpv, lo, ln, cap), want_all=True))
    ref = orc.pyramid(L, R, D, levels=1, num_paths=8, tau=tau, bands=(lo, ln, cap))[0]
    np.testing.assert_array_equal(raw, ref.dl)
    np.testing.assert_array_equal(dr, ref.dr)
    np.testing.assert_array_equal(d, ref.out)


@pytest.mark.parametrize("w,h,D,levels,R,P", [
    (160, 96, 64, 3, 4, 8), (97, 61, 48, 2, 4, 4), (130, 70, 128, 3, 2, 8), (64, 40, 32, 3, 64, 8),
    (200, 120, 256, 3, 4, 4), (50, 30, 40, 4, 4, 2), (23, 11, 16, 3, 4, 8), (8, 8, 8, 4, 1, 1),
])
def test_fused_pyramid(mpv, orc, w, h, D, levels, R, P):
    _log("pyramid", w, h, D, levels, R, P)
    L, Rt = _scene_pair(w + h + D, w, h, D - 1, ground=True)
    p = mpv.MPVParams(num_disp=D, num_paths=P)
    pyr = mpv.pyramid(_cuda(L), _cuda(Rt), p, levels=levels, radius=R, keep_levels=True)
    ref = orc.pyramid(L, Rt, D, levels=levels, radius=R, num_paths=P)
    for l in range(levels):
        np.testing.assert_array_equal(_np(pyr.level_raw[l]), ref[l].dl, err_msg=f"level {l}")
    np.testing.assert_array_equal(_np(pyr.raw), ref[-1].dl)
    np.testing.assert_array_equal(_np(pyr.right), ref[-1].dr)
    np.testing.assert_array_equal(_np(pyr.disp), ref[-1].out)


@pytest.mark.parametrize("name", ["c1", "c2", "c2p"])
def test_workload_parity_full_size(mpv, orc, name):
    """The measured workloads at their full sizes, in the launch configuration the benchmark
    times: every output pixel against the oracle."""
    from paper_2001_09678_amd.scene import config_scene
    sc, cfg = config_scene(name)
    _log("workload", name)
    p = mpv.MPVParams(num_disp=cfg["num_disp"], num_paths=cfg["num_paths"])
    pyr = mpv.pyramid(_cuda(sc.left), _cuda(sc.right), p, levels=cfg["levels"], radius=4, keep_levels=True)
    ref = orc.pyramid(sc.left, sc.right, cfg["num_disp"], levels=cfg["levels"], radius=4,
                      num_paths=cfg["num_paths"])
    for l in range(cfg["levels"]):
        np.testing.assert_array_equal(_np(pyr.level_raw[l]), ref[l].dl, err_msg=f"level {l}")
    np.testing.assert_array_equal(_np(pyr.disp), ref[-1].out)
    np.testing.assert_array_equal(_np(pyr.right), ref[-1].dr)


def test_repeatable_bits(mpv):
    """Same inputs twice give identical bits (no order-dependent arithmetic)."""
    from paper_2001_09678_amd.scene import config_scene
    sc, cfg = config_scene("c1")
    p = mpv.MPVParams(num_disp=64, num_paths=4)
    a = _np(mpv.pyramid(_cuda(sc.left), _cuda(sc.right), p, levels=1).disp).copy()
    b = _np(mpv.pyramid(_cuda(sc.left), _cuda(sc.right), p, levels=1).disp)
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("merge,sigma", [("sum", 0), ("layered_occ", 16)])
def test_paper_scope_full_size(mpv, orc, merge, sigma):
    """The paper's search scope (a quarter of the full range at every level below the top,
    Section 3.4 eqs. Ot1/Ot2: here radius D/8, 33 of 128 disparities) on the 1280x720
    workload, every output pixel against the oracle."""
    from paper_2001_09678_amd.scene import config_scene
    sc, cfg = config_scene("c2")
    _log("paper scope", merge, sigma)
    p = mpv.MPVParams(num_disp=128, num_paths=8, merge=merge, grad_sigma=sigma)
    pyr = mpv.pyramid(_cuda(sc.left), _cuda(sc.right), p, levels=3, radius=16, keep_levels=True)
    kw = dict(merge="sum") if merge == "sum" else dict(merge="layered", occ=True)
    ref = orc.pyramid(sc.left, sc.right, 128, levels=3, radius=16, num_paths=8, grad_sigma=sigma, **kw)
    for l in range(3):
        np.testing.assert_array_equal(_np(pyr.level_raw[l]), ref[l].dl, err_msg=f"level {l}")
    np.testing.assert_array_equal(_np(pyr.disp), ref[-1].out)
