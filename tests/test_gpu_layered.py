"""Layered path merge (Section 3.2: hierarchical merging, Table alg) on the HIP path vs the
CPU oracle, bit-exact, through the C ABI.

Every layer's scans run on the GPU (the first from the census, the later ones from the
merge of the previous layer's two partial volumes), the reduce decides on the last merge.
Both modes: the plain layered merge and the one with the occlusion strategy (the
left-to-right pass pays twice for disparity increases).
Compared: the raw WTA, the right disparity and the LR-checked map of single levels (full
range under every lane layout, fixed and variable bands, the masked full-range kernel for
wide bands), of pyramids (every level's raw WTA), of random configurations, and of the
full 1280x720 workloads."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

MERGES = ["layered", "layered_occ"]


def _orc(merge):
    """Oracle arguments of a merge mode: the layered merge, with the occlusion weight."""
    return dict(merge="layered", occ=merge == "layered_occ")


@pytest.fixture(scope="module")
def mpv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2001_09678_amd import mpv as m, _lib
    _lib.lib()
    return m


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _scene(seed, w, h, dmax, ground=False):
    from paper_2001_09678_amd.scene import make_scene
    s = make_scene(seed, w, h, dmax, 6, ground=ground)
    return s.left, s.right


def _log(*a):
    print(*a, flush=True)


def _check_level(got, ref):
    d, dr, raw = (_np(t) for t in got)
    np.testing.assert_array_equal(raw, ref.dl)
    np.testing.assert_array_equal(dr, ref.dr)
    np.testing.assert_array_equal(d, ref.out)


FULL_CASES = [
    # w, h, D, P, lambda, tau
    (33, 17, 5, 8, 8, 4), (70, 45, 64, 8, 8, 4), (129, 66, 100, 8, 8, 4), (61, 29, 128, 8, 8, 4),
    (37, 23, 200, 4, 8, 4), (30, 20, 256, 8, 8, 4), (40, 20, 32, 2, 8, 4), (1, 1, 4, 8, 8, 4),
    (5, 70, 16, 8, 8, 4), (70, 3, 16, 8, 8, 4),
    (45, 31, 32, 8, 8, 1),    # Potts
    (45, 31, 20, 8, 5, 2),
    (53, 41, 64, 8, 6, 3),    # runtime tau
    (45, 31, 20, 8, 3, 40),   # tau >= D: untruncated TV
    (40, 20, 17, 8, 0, 4),    # lambda = 0
]


@pytest.mark.parametrize("merge", MERGES)
@pytest.mark.parametrize("w,h,D,P,lam,tau", FULL_CASES)
def test_layered_match_full_range(mpv, orc, w, h, D, P, lam, tau, merge):
    _log("layered match", w, h, D, P, lam, tau, merge)
    L, R = _scene(w * 5 + D, w, h, max(D - 1, 0))
    p = mpv.MPVParams(num_disp=D, num_paths=P, lam=lam, tau=tau, merge=merge)
    ref = orc.pyramid(L, R, D, levels=1, num_paths=P, lam=lam, tau=tau, **_orc(merge))[0]
    _check_level(mpv.match(_cuda(L), _cuda(R), p, want_all=True), ref)


@pytest.mark.parametrize("merge", MERGES)
@pytest.mark.parametrize("full_lanes", [16, 32, 64])
@pytest.mark.parametrize("wpb", [1, 4])
def test_layered_lane_layouts(mpv, orc, full_lanes, wpb, merge):
    """Every full-range lane layout (2 packed pairs per lane where the range allows) and
    block shape gives the oracle's result."""
    w, h, D = 77, 39, 64
    _log("layered layout", full_lanes, wpb, merge)
    L, R = _scene(900 + full_lanes, w, h, D - 1)
    p = mpv.MPVParams(num_disp=D, num_paths=8, merge=merge)
    pyr = mpv.pyramid(_cuda(L), _cuda(R), p, levels=1, sched=mpv.Schedule(wpb, full_lanes, 0, 0))
    ref = orc.pyramid(L, R, D, levels=1, num_paths=8, **_orc(merge))[0]
    np.testing.assert_array_equal(_np(pyr.raw), ref.dl)
    np.testing.assert_array_equal(_np(pyr.right), ref.dr)
    np.testing.assert_array_equal(_np(pyr.disp), ref.out)


@pytest.mark.parametrize("cap,varlen,lam,tau", [
    (9, False, 8, 4), (16, True, 8, 4), (40, True, 8, 4), (60, True, 8, 4), (5, True, 8, 1),
    (12, False, 2, 9), (7, True, 6, 3)])
@pytest.mark.parametrize("merge", MERGES)
def test_layered_match_banded(mpv, orc, cap, varlen, lam, tau, merge):
    _log("layered banded", cap, varlen, lam, tau, merge)
    w, h, D = 91, 47, 96
    L, R = _scene(cap + 300, w, h, D - 1)
    rng = np.random.default_rng(cap + 7)
    lo = rng.integers(0, D - cap + 1, size=(h, w)).astype(np.int16)
    ln = rng.integers(1, cap + 1, size=(h, w)).astype(np.uint8) if varlen else None
    p = mpv.MPVParams(num_disp=D, num_paths=8, lam=lam, tau=tau, merge=merge)
    band = mpv.Band(_cuda(lo), cap, None if ln is None else _cuda(ln))
    ref = orc.pyramid(L, R, D, levels=1, num_paths=8, lam=lam, tau=tau, bands=(lo, ln, cap), **_orc(merge))[0]
    _check_level(mpv.match(_cuda(L), _cuda(R), p, band, want_all=True), ref)


@pytest.mark.parametrize("w,h,D,levels,R,P", [
    (160, 96, 64, 3, 4, 8), (97, 61, 48, 2, 4, 4), (130, 70, 128, 3, 2, 8), (64, 40, 32, 3, 64, 8),
    (200, 120, 256, 3, 4, 4), (50, 30, 40, 4, 4, 2), (23, 11, 16, 3, 4, 8),
])
@pytest.mark.parametrize("merge", MERGES)
def test_layered_pyramid(mpv, orc, w, h, D, levels, R, P, merge):
    _log("layered pyramid", w, h, D, levels, R, P, merge)
    L, Rt = _scene(w + h + D + 1, w, h, D - 1, ground=True)
    p = mpv.MPVParams(num_disp=D, num_paths=P, merge=merge)
    pyr = mpv.pyramid(_cuda(L), _cuda(Rt), p, levels=levels, radius=R, keep_levels=True)
    ref = orc.pyramid(L, Rt, D, levels=levels, radius=R, num_paths=P, **_orc(merge))
    for l in range(levels):
        np.testing.assert_array_equal(_np(pyr.level_raw[l]), ref[l].dl, err_msg=f"level {l}")
    np.testing.assert_array_equal(_np(pyr.right), ref[-1].dr)
    np.testing.assert_array_equal(_np(pyr.disp), ref[-1].out)


def _draw(seed):
    rng = np.random.default_rng([seed, 91])
    levels = int(rng.integers(1, 4))
    w = int(rng.integers(8 << (levels - 1), 180))
    h = int(rng.integers(4 << (levels - 1), 80))
    D = int(rng.choice([1, 3, 16, 31, 64, 97, 128, 200, 256]))
    P = int(rng.choice([2, 4, 8]))
    merge = MERGES[seed % 2]
    tau = int(rng.choice([1, 2, 3, 4, 6, 300]))
    te = max(1, min(tau, D - 1))
    layers = max(P // 2, 2 if merge == "layered_occ" else 1)
    lam = int(rng.integers(0, 231 // (layers * te) + 1))
    R = int(rng.choice([0, 1, 2, 4, 7]))
    sched = (int(rng.choice([1, 2, 4])), int(rng.choice([0, 32])), int(rng.choice([0, 32])), 0)
    return dict(levels=levels, w=w, h=h, D=D, P=P, tau=tau, lam=lam, R=R, sched=sched, merge=merge,
                seed=int(rng.integers(1, 10**6)))


@pytest.mark.parametrize("seed", range(24))
def test_layered_random(mpv, orc, seed):
    c = _draw(seed)
    _log("layered random", seed, c)
    L, Rt = _scene(c["seed"], c["w"], c["h"], max(c["D"] - 1, 0), ground=True)
    p = mpv.MPVParams(num_disp=c["D"], num_paths=c["P"], lam=c["lam"], tau=c["tau"], merge=c["merge"])
    pyr = mpv.pyramid(_cuda(L), _cuda(Rt), p, levels=c["levels"], radius=c["R"], keep_levels=True,
                      sched=mpv.Schedule(*c["sched"]))
    ref = orc.pyramid(L, Rt, c["D"], levels=c["levels"], radius=c["R"], num_paths=c["P"], lam=c["lam"],
                      tau=c["tau"], **_orc(c["merge"]))
    for l in range(c["levels"]):
        np.testing.assert_array_equal(_np(pyr.level_raw[l]), ref[l].dl, err_msg=f"level {l}")
    np.testing.assert_array_equal(_np(pyr.right), ref[-1].dr)
    np.testing.assert_array_equal(_np(pyr.disp), ref[-1].out)


@pytest.mark.parametrize("name,merge", [("c2", "layered"), ("c2p", "layered"), ("c2", "layered_occ"),
                                        ("c2p", "layered_occ")])
def test_layered_full_size(mpv, orc, name, merge):
    """The 1280x720, D=128 pair (multi-scale and plain full range), every output pixel
    against the oracle."""
    from paper_2001_09678_amd.scene import config_scene
    sc, cfg = config_scene(name)
    _log("layered workload", name, merge)
    p = mpv.MPVParams(num_disp=cfg["num_disp"], num_paths=cfg["num_paths"], merge=merge)
    pyr = mpv.pyramid(_cuda(sc.left), _cuda(sc.right), p, levels=cfg["levels"], radius=4, keep_levels=True)
    ref = orc.pyramid(sc.left, sc.right, cfg["num_disp"], levels=cfg["levels"], radius=4,
                      num_paths=cfg["num_paths"], **_orc(merge))
    for l in range(cfg["levels"]):
        np.testing.assert_array_equal(_np(pyr.level_raw[l]), ref[l].dl, err_msg=f"level {l}")
    np.testing.assert_array_equal(_np(pyr.right), ref[-1].dr)
    np.testing.assert_array_equal(_np(pyr.disp), ref[-1].out)


@pytest.mark.parametrize("merge", MERGES)
def test_layered_batch(mpv, orc, merge):
    """Eight pairs of their own sizes and ranges in one batch, run eagerly and replayed as a
    graph twice: each output equals the oracle's layered pyramid of that pair."""
    from paper_2001_09678_amd.scene import make_scene
    rng = np.random.default_rng(7000 + len(merge))
    levels, R, P = 3, 4, 8
    host, pairs = [], []
    for i in range(8):
        w, h = int(rng.integers(32, 170)), int(rng.integers(16, 90))
        D = int(rng.choice([16, 48, 64, 128, 256]))
        sc = make_scene(7100 + i, w, h, D - 1, 5, ground=True)
        host.append((sc.left, sc.right, D))
        pairs.append((_cuda(sc.left), _cuda(sc.right), D))
    _log("layered batch", merge, [(l.shape, D) for l, _, D in host])
    b = mpv.Batch(pairs, mpv.MPVParams(num_disp=128, num_paths=P, merge=merge), levels, R, want_all=True)
    refs = [orc.pyramid(l, r, D, levels=levels, radius=R, num_paths=P, **_orc(merge))[-1] for l, r, D in host]
    for run in ("run", "run_graph", "run_graph"):
        getattr(b, run)()
        for i, ref in enumerate(refs):
            np.testing.assert_array_equal(_np(b.raw[i]), ref.dl, err_msg=f"{run} pair {i}")
            np.testing.assert_array_equal(_np(b.right[i]), ref.dr, err_msg=f"{run} pair {i}")
            np.testing.assert_array_equal(_np(b.disp[i]), ref.out, err_msg=f"{run} pair {i}")
    b.close()
