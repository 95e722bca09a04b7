"""Pins of the float64 warm-start network reference (oracle.warmnet)."""

import numpy as np
import pytest

from oracle import warmnet as wn


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_conv_matches_brute_force_loops():
    rng = _rng(1)
    x = rng.standard_normal((2, 5, 6, 3))
    w = rng.standard_normal((3, 3, 3, 4))
    b = rng.standard_normal(4)
    got = wn.conv3x3(x, w, b)
    n, h, wd, ci = x.shape
    ref = np.zeros((n, h, wd, 4))
    for a in range(n):
        for y in range(h):
            for xx in range(wd):
                for co in range(4):
                    s = b[co]
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            for c in range(ci):
                                s += x[a, (y + dy) % h, (xx + dx) % wd, c] * w[dy + 1, dx + 1, c, co]
                    ref[a, y, xx, co] = s
    assert np.allclose(got, ref, rtol=0, atol=1e-12)


def test_conv_adjoints():
    """<conv(x), g> = <x, conv^T g> = <w, dW(x, g)> (the forward is linear in
    the input and in the weights)."""
    rng = _rng(2)
    x = rng.standard_normal((2, 8, 4, 3))
    w = rng.standard_normal((3, 3, 3, 5))
    g = rng.standard_normal((2, 8, 4, 5))
    lhs = float(np.sum(wn.conv3x3(x, w) * g))
    assert lhs == pytest.approx(float(np.sum(x * wn.conv3x3_grad_input(g, w))), rel=1e-12)
    assert lhs == pytest.approx(float(np.sum(w * wn.conv3x3_grad_weight(x, g))), rel=1e-12)


def test_resampling_adjoints_and_values():
    rng = _rng(3)
    x = rng.standard_normal((2, 8, 4, 3))
    y = rng.standard_normal((2, 4, 2, 3))
    assert float(np.sum(wn.pool2(x) * y)) == pytest.approx(float(np.sum(x * wn.pool2_adjoint(y))), rel=1e-12)
    z = rng.standard_normal((2, 16, 8, 3))
    assert float(np.sum(wn.up2(x) * z)) == pytest.approx(float(np.sum(x * wn.up2_adjoint(z))), rel=1e-12)
    # values: pooling averages a 2x2 block, upsampling copies it
    assert wn.pool2(x)[1, 2, 1, 2] == pytest.approx(x[1, 4:6, 2:4, 2].mean())
    assert np.all(wn.up2(y)[0, 2:4, 2:4, 1] == y[0, 1, 1, 1])


def test_conv_is_translation_equivariant_on_the_torus():
    rng = _rng(4)
    x = rng.standard_normal((1, 8, 8, 2))
    w = rng.standard_normal((3, 3, 2, 3))
    a = wn.conv3x3(np.roll(x, (3, -2), axis=(1, 2)), w)
    b = np.roll(wn.conv3x3(x, w), (3, -2), axis=(1, 2))
    assert np.allclose(a, b, atol=1e-12)


def test_network_gradient_matches_finite_differences():
    """Central differences of the loss for sampled entries of every weight
    and bias (float64, tiny network)."""
    ch = (3, 4, 4, 5)
    rng = _rng(5)
    p = wn.init_params(ch, seed=7)
    # a non-zero output layer and biases so every path carries gradient
    p.w[-1] = rng.standard_normal(p.w[-1].shape) * 0.3
    for b in p.b:
        b[:] = rng.standard_normal(b.shape) * 0.1
    x = rng.standard_normal((2, 16, 16, 4))
    tgt = rng.standard_normal((2, 16, 16))
    tp = wn.forward(p, x, ch)
    g = wn.backward(p, tp, tgt, ch)
    h = 1e-6
    for i in range(len(p.w)):
        for arr, garr in ((p.w, g.w), (p.b, g.b)):
            flat = arr[i].reshape(-1)
            for j in rng.choice(flat.size, size=min(3, flat.size), replace=False):
                old = flat[j]
                flat[j] = old + h
                lp = wn.loss(wn.forward(p, x, ch).y, tgt)
                flat[j] = old - h
                lm = wn.loss(wn.forward(p, x, ch).y, tgt)
                flat[j] = old
                fd = (lp - lm) / (2 * h)
                an = garr[i].reshape(-1)[j]
                assert an == pytest.approx(fd, rel=1e-5, abs=1e-9), (i, j)


def test_layer_shapes_and_zero_initial_prediction():
    ch = (32, 64, 96, 128)
    shapes = wn.layer_shapes(ch)
    assert len(shapes) == 15
    assert shapes[0] == (4, 32) and shapes[-1] == (32, 1)
    assert shapes[8] == (128, 96) and shapes[13] == (32, 32)
    p = wn.init_params((4, 4, 4, 4), seed=0)
    y = wn.forward(p, _rng(0).standard_normal((1, 16, 16, 4)), (4, 4, 4, 4)).y
    assert np.all(y == 0.0)


def test_features_scale_invariance_and_mask():
    rng = _rng(6)
    d = rng.standard_normal((16, 16)) * 30
    npix = np.exp(rng.standard_normal((16, 16))) * 50
    mask = (rng.random((16, 16)) > 0.2).astype(np.uint8)
    f, sig = wn.features(d, npix, mask)
    assert sig == pytest.approx(np.sqrt(npix[mask == 1].mean()))
    f2, sig2 = wn.features(3.0 * d, 9.0 * npix, mask)
    assert sig2 == pytest.approx(3.0 * sig)
    assert np.allclose(f, f2, atol=1e-12)
    assert np.all(f[mask == 0][:, :3] == 0.0)
    assert np.all(f[mask == 1, 2] == 1.0)
    # row channel: mean of the observed d / sigma of the row, on every pixel
    y = 5
    obs = mask[y] == 1
    assert np.allclose(f[y, :, 3], (d[y, obs] / sig).mean())


def test_adam_first_step_moves_by_lr_times_sign():
    """With zero moments the bias-corrected first step is lr g / (|g| + eps)."""
    p = wn.Params([np.array([[1.0, -2.0]])], [np.array([0.5])])
    g = wn.Params([np.array([[3.0, -1e-3]])], [np.array([0.0])])
    opt = wn.Adam(lr=0.01)
    q = opt.step(p, g)
    assert q.w[0][0, 0] == pytest.approx(1.0 - 0.01 * 3.0 / (3.0 + 1e-8))
    assert q.w[0][0, 1] == pytest.approx(-2.0 + 0.01 * 1e-3 / (1e-3 + 1e-8))
    assert q.b[0][0] == 0.5
