"""Pins of the CPU reference of the band-proposal network (oracle/cnn.py).

* the convolution against an explicit loop over taps and channels;
* the whole backward pass (network + heads + loss) against central finite differences in
  float64, for weights, biases and inputs;
* features against a direct per-pixel evaluation of their definitions;
* heads/bands on hand-worked values; bfloat16 rounding on hand-picked bit patterns.
"""
import numpy as np
import pytest

from oracle import cnn


def test_conv_matches_explicit_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 4, 5, 3))
    w = rng.normal(size=(3, 3, 3, 2))
    b = rng.normal(size=2)
    y = cnn.conv3x3(x, w, b)
    for n in range(2):
        for i in range(4):
            for j in range(5):
                for d in range(2):
                    s = b[d]
                    for ky in range(3):
                        for kx in range(3):
                            yi, xj = i + ky - 1, j + kx - 1
                            if 0 <= yi < 4 and 0 <= xj < 5:
                                s += sum(x[n, yi, xj, c] * w[ky, kx, c, d] for c in range(3))
                    assert y[n, i, j, d] == pytest.approx(s, abs=1e-12)


def _total_loss(x, weights, dl, labels, beta):
    acts = cnn.forward(x, weights)
    return cnn.loss_and_grad(acts[-1], dl, labels, beta)[0]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    N, Hc, Wc = 2, 3, 4
    chans = [4, 5, 3]
    weights = [(rng.normal(0, 0.4, (3, 3, a, b)), rng.normal(0, 0.1, b)) for a, b in zip(chans[:-1], chans[1:])]
    # bias the heads into their linear ranges
    weights[-1][1][:] = [0.3, 5.0, 0.5]
    x = rng.normal(size=(N, Hc, Wc, chans[0]))
    dl = rng.integers(0, 10, size=(N, Hc, Wc)).astype(np.float64)
    labels = (4 * dl.repeat(4, 1).repeat(4, 2) + rng.integers(-6, 7, size=(N, 4 * Hc, 4 * Wc))).astype(np.int64)
    labels[rng.random(labels.shape) < 0.2] = -1
    beta = 0.05
    acts = cnn.forward(x, weights)
    _, g, count = cnn.loss_and_grad(acts[-1], dl, labels, beta)
    assert count > 0
    grads, dx = cnn.backward(acts, weights, g)
    h = 1e-6
    checked = 0
    for li, (w, b) in enumerate(weights):
        for arr, garr in ((w, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = _total_loss(x, weights, dl, labels, beta)
                flat[idx] = old - h
                lm = _total_loss(x, weights, dl, labels, beta)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                an = garr.reshape(-1)[idx]
                assert an == pytest.approx(fd, rel=1e-6, abs=1e-9), (li, idx)
                checked += 1
    flat = x.reshape(-1)
    for idx in rng.choice(flat.size, size=12, replace=False):
        old = flat[idx]
        flat[idx] = old + h
        lp = _total_loss(x, weights, dl, labels, beta)
        flat[idx] = old - h
        lm = _total_loss(x, weights, dl, labels, beta)
        flat[idx] = old
        assert dx.reshape(-1)[idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-9)
        checked += 1
    assert checked >= 40


def test_features_match_definition(orc):
    rng = np.random.default_rng(2)
    H, W, D0 = 5, 7, 6
    S = rng.integers(0, 300, size=(H, W, D0)).astype(np.int64)
    img = rng.integers(0, 256, size=(H, W)).astype(np.uint8)
    dl, _, out = orc.wta_lr(S, D0, 1)
    f = cnn.features(img, dl, out, S, 8, 8, 4)
    Z = 8 * (24 + 8 * 4)
    for y in range(H):
        for x in range(W):
            s = S[y, x] - S[y, x].min()
            d = int(dl[y, x])
            assert s[d] == 0
            expect = [img[y, x] / 255, d / D0, float(out[y, x] >= 0),
                      s[max(d - 1, 0)] / Z, s[min(d + 1, D0 - 1)] / Z,
                      s[max(d - 2, 0)] / Z, s[min(d + 2, D0 - 1)] / Z]
            far = [s[k] for k in range(D0) if abs(k - d) > 1]
            expect.append(min(far) / Z if far else 1.0)
            np.testing.assert_allclose(f[y, x], expect, rtol=0, atol=1e-15)


def test_heads_and_bands_hand_example():
    o = np.array([[[[1.4, 3.5, 0.7], [-0.6, -2.0, 0.2], [0.5, 20.0, 1.5]]]])  # [1,1,3,3]
    dl = np.array([[[10, 0, 31]]])
    c, w, conf = cnn.heads(o, dl)
    np.testing.assert_allclose(c[0, 0], [41.4, -0.6, 124.5])
    np.testing.assert_allclose(w[0, 0], [5.5, 2.0, 16.0])
    np.testing.assert_allclose(conf[0, 0], [0.7, 0.2, 1.0])
    lo, ln, low = cnn.bands(o[0], dl[0], 12, 4, 128, 0.5)
    # pixel 0: center round(41.4)=41, width 2+round(3.5)=6 -> lo 38
    # pixel 1: conf 0.2 < 0.5 -> width 16, center round(-0.6) = -1 -> lo clamp(-9)=0
    # pixel 2: center round(124.5)=125, width 2+14=16 -> lo clamp(117, 0, 112)=112
    assert low == 1
    assert lo[0, :4].tolist() == [38] * 4 and ln[0, 0] == 6
    assert lo[3, 4] == 0 and ln[3, 4] == 16
    assert lo[2, 8] == 112 and ln[2, 11] == 16


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.0e-5])
    r = cnn.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0            # exactly half an ulp above 1: ties to even (mantissa 0)
    assert r[2] == 1.0 + 2 ** -7  # above half: rounds up
    assert r[3] == -2.5
    assert abs(r[4] - 3.0e-5) / 3.0e-5 < 2 ** -8
