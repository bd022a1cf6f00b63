"""Learned band proposal on the GPU vs the CPU reference (oracle/cnn.py), through the C ABI.

Layer-local parity with identical BF16 inputs: forward relative L2 <= 1e-3 (only the FP32
accumulation order differs), backward (dX, dW, db) <= 1e-2. Features and band maps are
integer/rounding decisions taken in the kernel's precision and must match exactly.
Training: the loss falls and save + resume continues bit-identically. The learned
matcher's finest level equals the oracle run on the same band map.
"""
import numpy as np
import pytest

from oracle import cnn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2001_09678_amd import learned, _lib
    _lib.lib()
    return learned


def _log(*a):
    print(*a, flush=True)


def _bf16_bits(a):
    """float64 -> bf16 bit patterns (int16) with round-to-nearest-even."""
    f = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return (((f + 0x7FFF + ((f >> 16) & 1)) >> 16).astype(np.uint16)).view(np.int16)


def _bits_to_f(b):
    return (np.asarray(b).view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _pack(lb, w, cin, cout):
    import torch
    from paper_2001_09678_amd import _lib as L
    lib = L.lib()
    wf = torch.empty(int(lib.mpv_lb_packed_elems(cin, cout)), dtype=torch.int16, device="cuda")
    wb = torch.empty(int(lib.mpv_lb_packed_bwd_elems(cin, cout)), dtype=torch.int16, device="cuda")
    wt = _cuda(w.astype(np.float32).reshape(-1))
    L.check(lib.mpv_lb_pack(lb._p(wt), cin, cout, lb._p(wf), lb._p(wb), lb._s()), "pack")
    return wf, wb


@pytest.mark.parametrize("cin,cout,relu", [(8, 32, 1), (32, 32, 1), (32, 3, 0)])
def test_conv_forward(lb, cin, cout, relu):
    import torch
    from paper_2001_09678_amd import _lib as L
    _log("conv fwd", cin, cout)
    rng = np.random.default_rng(cin + cout)
    n, h, w = 2, 11, 37
    x = _bf16_bits(rng.normal(size=(n, h, w, cin)))
    wt = rng.normal(0, np.sqrt(2 / (9 * cin)), (3, 3, cin, cout))
    b = rng.normal(0, 0.1, cout)
    wf, _ = _pack(lb, wt, cin, cout)
    y = torch.empty((n, h, w, 4 if cout == 3 else cout), dtype=torch.float32, device="cuda")
    bt = _cuda(b.astype(np.float32))
    xg = _cuda(x)
    L.check(L.lib().mpv_lb_conv(lb._p(xg), n, h, w, cin, lb._p(wf), lb._p(bt), cout, relu, None, 0,
                                lb._p(y), y.shape[-1], 1, lb._s()), "conv")
    ref = cnn.conv3x3(_bits_to_f(x), cnn.bf16_round(wt), b.astype(np.float32).astype(np.float64))
    if relu:
        ref = np.maximum(ref, 0)
    got = _np(y)
    assert _rel(got[..., :cout], ref) <= 1e-3
    if y.shape[-1] > cout:
        assert (got[..., cout:] == 0).all()


@pytest.mark.parametrize("cin,cout", [(32, 32), (32, 3)])
def test_conv_backward_data_and_weights(lb, cin, cout):
    import torch
    from paper_2001_09678_amd import _lib as L
    _log("conv bwd", cin, cout)
    lib = L.lib()
    rng = np.random.default_rng(7 + cout)
    n, h, w = 2, 13, 29
    c4 = (cout + 3) // 4 * 4
    x = _bf16_bits(rng.normal(size=(n, h, w, cin)))
    dzf = np.zeros((n, h, w, c4))
    dzf[..., :cout] = rng.normal(size=(n, h, w, cout))
    dz = _bf16_bits(dzf)
    wt = rng.normal(0, 0.2, (3, 3, cin, cout))
    _, wb = _pack(lb, wt, cin, cout)
    xg, dzg = _cuda(x), _cuda(dz)  # held: a temporary's block would be reused by the next one
    dx = torch.empty((n, h, w, cin), dtype=torch.float32, device="cuda")
    L.check(lib.mpv_lb_conv(lb._p(dzg), n, h, w, c4, lb._p(wb), None, cin, 0, None, 0, lb._p(dx), cin, 1,
                            lb._s()), "conv bwd-data")
    rdx, rdw, rdb = cnn.conv3x3_backward(_bits_to_f(x), cnn.bf16_round(wt), _bits_to_f(dz)[..., :cout])
    assert _rel(_np(dx), rdx) <= 1e-2
    dw = torch.empty(9 * cin * cout, dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    need = int(lib.mpv_lb_dw_workspace_bytes(n, h, w, cin, cout))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    L.check(lib.mpv_lb_conv_dw(lb._p(xg), lb._p(dzg), c4, n, h, w, cin, cout, lb._p(dw), lb._p(db),
                               lb._p(ws), need, lb._s()), "conv dw")
    assert _rel(_np(dw).reshape(3, 3, cin, cout), rdw) <= 1e-2
    assert _rel(_np(db), rdb) <= 1e-2
    # fixed-order reductions: a second run gives the same bits
    dw2 = torch.empty_like(dw)
    L.check(lib.mpv_lb_conv_dw(lb._p(xg), lb._p(dzg), c4, n, h, w, cin, cout, lb._p(dw2), lb._p(db),
                               lb._p(ws), need, lb._s()), "conv dw")
    assert torch.equal(dw, dw2)


def test_loss_and_heads(lb):
    _log("loss")
    rng = np.random.default_rng(3)
    n, hc, wc = 2, 9, 14
    H, W = 4 * hc + 2, 4 * wc + 3
    o = np.zeros((n, hc, wc, 4), np.float32)
    o[..., 0] = rng.normal(0, 3, (n, hc, wc))
    o[..., 1] = rng.uniform(-2, 16, (n, hc, wc))
    o[..., 2] = rng.uniform(-0.3, 1.3, (n, hc, wc))
    raw = rng.integers(0, 32, (n, hc, wc)).astype(np.int16)
    lab = rng.integers(0, 128, (n, H, W)).astype(np.int16)
    up = np.repeat(np.repeat(4 * raw.astype(np.int64), 4, 1), 4, 2)
    lab[:, :4 * hc, :4 * wc] = (up + rng.integers(-8, 9, up.shape)).clip(0, 127)
    lab[rng.random(lab.shape) < 0.1] = -1
    count = int((lab[:, :4 * hc, :4 * wc] >= 0).sum())
    dz, parts = lb.loss(_cuda(o), _cuda(raw), _cuda(lab), 0.05, 1.0 / count)
    rl, rg, rc = cnn.loss_and_grad(o[..., :3].astype(np.float64), raw.astype(np.float64), lab, 0.05)
    assert rc == count
    assert float(_np(parts).sum()) == pytest.approx(rl, rel=1e-4)
    got = _bits_to_f(_np(dz))
    assert _rel(got[..., :3], rg) <= 1e-2
    assert (got[..., 3] == 0).all()


def test_features_exact(lb, orc):
    """Coarse features equal the oracle's (same decisions, bf16 rounding of the same FP32
    quotients) on a 160x90 coarse pair, D=32, 8 paths."""
    from paper_2001_09678_amd import mpv
    from paper_2001_09678_amd.scene import make_scene
    _log("features")
    sc = make_scene(41, 640, 360, 127, 25, ground=True)
    L0, R0 = orc.downsample(orc.downsample(sc.left)), orc.downsample(orc.downsample(sc.right))
    params = mpv.MPVParams(num_disp=32, num_paths=8)
    co = lb.Coarse(params, L0.shape[1], L0.shape[0])
    feat, raw, disp = co(_cuda(L0), _cuda(R0))
    ref = orc.pyramid(L0, R0, 32, levels=1, num_paths=8, keep_sums=True)[0]
    np.testing.assert_array_equal(_np(raw), ref.dl)
    np.testing.assert_array_equal(_np(disp), ref.out)
    rf = cnn.features(L0, ref.dl, ref.out, ref.S, 8, 8, 4)
    np.testing.assert_array_equal(_np(feat).view(np.uint16), _bf16_bits(rf).view(np.uint16))


def test_bands_exact(lb):
    """Band maps from the network output, recomputed here in FP32 (the kernel's precision)."""
    _log("bands")
    rng = np.random.default_rng(5)
    hc, wc, H, W, D = 11, 17, 46, 70, 128
    o = np.zeros((hc, wc, 4), np.float32)
    o[..., 0] = rng.normal(0, 4, (hc, wc)).astype(np.float32)
    o[..., 0][0, :4] = [0.5, -0.5, 1.5, 2.5]          # exact halves
    o[..., 1] = rng.uniform(-3, 18, (hc, wc)).astype(np.float32)
    o[..., 1][1, :3] = [3.5, 4.5, -0.5]
    o[..., 2] = rng.uniform(-0.5, 1.5, (hc, wc)).astype(np.float32)
    raw = rng.integers(0, 33, (hc, wc)).astype(np.int16)
    lo, ln, nlow = lb.bands(_cuda(o), _cuda(raw), W, H, D, 0.5)
    f32 = np.float32
    center = f32(4) * raw.astype(f32) + o[..., 0]
    ci = np.floor(center + f32(0.5)).astype(np.int64)
    w = 2 + np.clip(np.floor(o[..., 1] + f32(0.5)), 0, 14).astype(np.int64)
    low = o[..., 2] < f32(0.5)
    w = np.minimum(np.where(low, 16, w), D)
    rlo = np.clip(ci - w // 2, 0, D - w)
    fy = np.minimum(np.arange(H) // 4, hc - 1)
    fx = np.minimum(np.arange(W) // 4, wc - 1)
    np.testing.assert_array_equal(_np(lo), rlo[fy][:, fx])
    np.testing.assert_array_equal(_np(ln), w[fy][:, fx])
    assert int(_np(nlow)[0]) == int(low.sum())
    # the float64 reference agrees except where FP32 rounding moves a half-way case
    rlo64, rln64, rlow64 = cnn.bands(o[..., :3].astype(np.float64), raw, W, H, D, 0.5)
    assert (rlo64 == _np(lo)).mean() > 0.999 and rlow64 == int(low.sum())


def test_network_gradients_vs_reference(lb):
    """Whole network, identical BF16 inputs and weights: every parameter gradient within
    1e-2 relative L2 of the float64 reference."""
    import torch
    _log("network gradients")
    rng = np.random.default_rng(11)
    n, hc, wc = 2, 12, 20
    H, W = 4 * hc, 4 * wc
    net = lb.BandNet("cuda", seed=3)
    feat = _bf16_bits(np.abs(rng.normal(0.3, 0.3, (n, hc, wc, 8))))
    raw = rng.integers(0, 32, (n, hc, wc)).astype(np.int16)
    up = np.repeat(np.repeat(4 * raw.astype(np.int64), 4, 1), 4, 2)
    lab = (up + rng.integers(-6, 7, up.shape)).clip(0, 127).astype(np.int16)
    count = int((lab >= 0).sum())
    o, acts = net.forward(_cuda(feat))
    dz, _ = lb.loss(o, _cuda(raw), _cuda(lab), 0.05, 1.0 / count)
    net.backward(acts, dz)
    params = _np(net.params).astype(np.float64)
    weights = []
    for i, (ci, co) in enumerate(net.layers):
        wo, bo = net.offsets[i]
        weights.append((cnn.bf16_round(params[wo:bo].reshape(3, 3, ci, co)), params[bo:bo + co].astype(np.float32).astype(np.float64)))
    # reference forward in float64 from the same bf16 input; activations rounded to bf16 like the GPU
    x = _bits_to_f(feat)
    ra = [x]
    for i, (w, b) in enumerate(weights):
        z = cnn.conv3x3(ra[-1], w, b)
        ra.append(cnn.bf16_round(np.maximum(z, 0)) if i + 1 < len(weights) else z)
    _, g, _ = cnn.loss_and_grad(ra[-1][..., :3], raw.astype(np.float64), lab, 0.05)
    grads, _ = cnn.backward(ra, weights, g)
    got = _np(net.grad).astype(np.float64)
    for i, (ci, co) in enumerate(net.layers):
        wo, bo = net.offsets[i]
        assert _rel(got[wo:bo].reshape(3, 3, ci, co), grads[i][0]) <= 1e-2, f"dW layer {i}"
        assert _rel(got[bo:bo + co], grads[i][1]) <= 1e-2, f"db layer {i}"


@pytest.fixture(scope="module")
def small_data(lb):
    from paper_2001_09678_amd import mpv
    specs = lb.scene_specs(90000, 6, width=320, height=192, num_disp=64)
    return lb.Dataset(specs, mpv.MPVParams(num_disp=64, num_paths=8), workers=6)


def test_training_loss_falls_and_resume_is_exact(lb, small_data, tmp_path):
    import torch
    _log("training")
    net = lb.BandNet("cuda", seed=1)
    before = lb.dataset_loss(net, small_data)
    lb.train(net, small_data, steps=300, batch=4, lr=2e-3, seed=5, log_every=50, log=_log)
    after = lb.dataset_loss(net, small_data)
    _log("dataset loss", before, "->", after)
    assert after < 0.9 * before
    # k steps straight == k/2 steps + save + resume + k/2 steps (bit for bit)
    a = lb.BandNet("cuda", seed=2)
    lb.train(a, small_data, steps=20, batch=4, seed=9, log_every=0)
    b = lb.BandNet("cuda", seed=2)
    ck = str(tmp_path / "ck.npz")
    lb.train(b, small_data, steps=10, batch=4, seed=9, log_every=0, ckpt=ck, ckpt_every=10)
    c, extra = lb.BandNet.load(ck)
    assert extra["step"] == 10 and c.step == 10
    lb.train(c, small_data, steps=20, batch=4, seed=9, start_step=10, rng_state=extra["rng"], log_every=0)
    assert torch.equal(a.params, c.params)
    assert torch.equal(a.m, c.m) and torch.equal(a.v, c.v)


def test_learned_matcher_bitexact_given_bands(lb, orc):
    """The learned matcher's finest level equals the oracle's Viterbi on the same band map."""
    from paper_2001_09678_amd import mpv
    from paper_2001_09678_amd.scene import make_scene
    _log("learned matcher")
    sc = make_scene(42001, 320, 192, 63, 12, ground=True)
    params = mpv.MPVParams(num_disp=64, num_paths=8)
    net = lb.BandNet("cuda", seed=4)
    m = lb.LearnedMatcher(net, params, 320, 192)
    L, R = _cuda(sc.left), _cuda(sc.right)
    out = m(L, R, allow_fallback=False)
    lo, ln = _np(m.lo), _np(m.len)
    ref = orc.pyramid(sc.left, sc.right, 64, levels=1, num_paths=8, bands=(lo, ln, 16))[0]
    np.testing.assert_array_equal(_np(out), ref.out)


def test_committed_weights_full_size(lb, orc):
    """Trained weights at 1280x720, D=128: the banded finest level equals the oracle's Viterbi
    on the GPU's band map; a frame forced to fall back equals plain full-range MPV."""
    import os
    from paper_2001_09678_amd import mpv
    from paper_2001_09678_amd.scene import make_scene
    _log("committed weights 1280x720")
    assert os.path.exists(lb.DEFAULT_WEIGHTS)
    net, meta = lb.BandNet.load(lb.DEFAULT_WEIGHTS)
    assert net.step == meta["steps"]
    sc = make_scene(42005, 1280, 720, 127, 30, ground=True)
    params = mpv.MPVParams(num_disp=128, num_paths=8)
    L, R = _cuda(sc.left), _cuda(sc.right)
    m = lb.LearnedMatcher(net, params, 1280, 720)
    out = m(L, R, allow_fallback=False)
    lo, ln = _np(m.lo), _np(m.len)
    assert ln.min() >= 2 and ln.max() <= 16
    ref = orc.pyramid(sc.left, sc.right, 128, levels=1, num_paths=8, bands=(lo, ln, 16))[0]
    np.testing.assert_array_equal(_np(out), ref.out)
    forced = lb.LearnedMatcher(net, params, 1280, 720, lb.LearnedConfig(fallback_frac=-1.0))
    got = forced(L, R)
    assert forced.last_fallback
    np.testing.assert_array_equal(_np(got), _np(mpv.match(L, R, params)))
