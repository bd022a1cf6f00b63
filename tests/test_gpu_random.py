"""Seeded random sweep: HIP path vs the CPU oracle, bit-exact, through the C ABI.

Each case draws its own shape (odd sizes, tails of every lane layout), disparity range,
levels, band radius, paths, lambda and tau (within the fused path's limits), scene and
schedule from a seeded generator, then compares the fused pyramid (every level's raw
winners, the right disparity and the LR-checked map), a single level with a random
variable-length band, and a small batch of such pairs against the oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N_CASES = 24


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


def _draw(seed):
    """One random configuration (fused limits: 24 + lambda*min(tau, D-1) <= 255)."""
    rng = np.random.default_rng([seed, 77])
    levels = int(rng.integers(1, 5))
    w = int(rng.integers(8 << (levels - 1), 200))
    h = int(rng.integers(4 << (levels - 1), 90))
    D = int(rng.choice([1, 3, 16, 31, 64, 97, 128, 200, 256]))
    P = int(rng.choice([1, 2, 4, 8]))
    tau = int(rng.choice([1, 2, 3, 4, 6, 300]))
    lam = int(rng.integers(0, 231 // max(1, min(tau, max(D - 1, 1))) + 1))
    R = int(rng.choice([0, 1, 2, 4, 7]))
    sched = (int(rng.choice([1, 2, 4])), int(rng.choice([0, 32])), int(rng.choice([0, 32])), 0)
    return dict(levels=levels, w=w, h=h, D=D, P=P, tau=tau, lam=lam, R=R, sched=sched,
                scene_seed=int(rng.integers(1, 10**6)))


def _pair(c):
    from paper_2001_09678_amd.scene import make_scene
    sc = make_scene(c["scene_seed"], c["w"], c["h"], max(c["D"] - 1, 0), 5, ground=True)
    return sc.left, sc.right


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_pyramid(mpv, orc, seed):
    c = _draw(seed)
    print("case", seed, c, flush=True)
    L, R = _pair(c)
    p = mpv.MPVParams(num_disp=c["D"], num_paths=c["P"], lam=c["lam"], tau=c["tau"])
    s = mpv.Schedule(*c["sched"])
    pyr = mpv.pyramid(_cuda(L), _cuda(R), p, levels=c["levels"], radius=c["R"], keep_levels=True, sched=s)
    ref = orc.pyramid(L, R, c["D"], levels=c["levels"], radius=c["R"], num_paths=c["P"], lam=c["lam"],
                      tau=c["tau"])
    for l in range(c["levels"]):
        np.testing.assert_array_equal(_np(pyr.level_raw[l]), ref[l].dl, err_msg=f"level {l}")
    np.testing.assert_array_equal(_np(pyr.right), ref[-1].dr)
    np.testing.assert_array_equal(_np(pyr.disp), ref[-1].out)


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_band_level(mpv, orc, seed):
    c = _draw(1000 + seed)
    print("case", seed, c, flush=True)
    L, R = _pair(c)
    D = c["D"]
    rng = np.random.default_rng(seed)
    cap = int(rng.integers(1, min(D, 40) + 1))
    lo = rng.integers(0, D - cap + 1, size=(c["h"], c["w"])).astype(np.int16)
    ln = rng.integers(1, cap + 1, size=(c["h"], c["w"])).astype(np.uint8)
    p = mpv.MPVParams(num_disp=D, num_paths=c["P"], lam=c["lam"], tau=c["tau"])
    band = mpv.Band(_cuda(lo), cap, _cuda(ln))
    d, r, raw = mpv.match(_cuda(L), _cuda(R), p, band, want_all=True)
    ref = orc.pyramid(L, R, D, levels=1, num_paths=c["P"], lam=c["lam"], tau=c["tau"], bands=(lo, ln, cap))[0]
    np.testing.assert_array_equal(_np(raw), ref.dl)
    np.testing.assert_array_equal(_np(r), ref.dr)
    np.testing.assert_array_equal(_np(d), ref.out)


def test_random_batch(mpv, orc):
    """Eight random pairs (own sizes and ranges, shared parameters) in one batch, graph
    replayed twice: each output equals the oracle."""
    rng = np.random.default_rng(4242)
    levels, R, P = 3, 4, 8
    pairs, host = [], []
    for i in range(8):
        w, h = int(rng.integers(32, 180)), int(rng.integers(16, 90))
        D = int(rng.choice([16, 48, 64, 128, 256]))
        from paper_2001_09678_amd.scene import make_scene
        sc = make_scene(5000 + i, w, h, D - 1, 5, ground=True)
        host.append((sc.left, sc.right, D))
        pairs.append((_cuda(sc.left), _cuda(sc.right), D))
    b = mpv.Batch(pairs, mpv.MPVParams(num_disp=128, num_paths=P), levels, R)
    for _ in range(2):
        b.run_graph()
        for (l, r, D), out in zip(host, b.disp):
            ref = orc.pyramid(l, r, D, levels=levels, radius=R, num_paths=P)[-1]
            np.testing.assert_array_equal(_np(out), ref.out)
    b.close()
