"""Pins of the U-Net oracle (the learned warm start; not part of the paper):
its convolution against scipy's 2-D correlation, the adjoint pairs, and its
hand-written backward pass against central finite differences."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import unet


def _params(width, levels, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout, *_ in unet.layer_table(width, levels):
        kpad = (9 * cin + 31) // 32 * 32
        w = np.zeros((cout, kpad))
        w[:, :9 * cin] = rng.normal(0, np.sqrt(2.0 / (9 * cin)), size=(cout, 9 * cin))
        parts += [w.ravel(), rng.normal(0, 0.05, size=cout)]
    parts += [rng.normal(0, np.sqrt(1.0 / width), size=width), [0.1]]
    return np.concatenate([np.ravel(p) for p in parts])


def test_conv3x3_is_scipy_correlation():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 7, 9, 3))
    W = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y = unet.conv3x3(x, W, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, :, :, c], W[o, :, :, c], mode="same") for c in range(3))
            np.testing.assert_allclose(y[n, :, :, o], ref, atol=1e-12)


def test_adjoint_pairs():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 8, 6, 3))
    y = rng.normal(size=(2, 4, 3, 3))
    assert np.sum(unet.pool(x) * y) == pytest.approx(np.sum(x * unet.pool_back(y)), rel=1e-12)
    z = rng.normal(size=(2, 8, 6, 3))
    assert np.sum(unet.up(y) * z) == pytest.approx(np.sum(y * unet.up_back(z)), rel=1e-12)
    # conv3x3_back's input gradient is the adjoint of the convolution without bias
    W = rng.normal(size=(5, 3, 3, 3))
    g = rng.normal(size=(2, 8, 6, 5))
    dx, _, _ = unet.conv3x3_back(x, W, g)
    assert np.sum(unet.conv3x3(x, W, np.zeros(5)) * g) == pytest.approx(np.sum(x * dx), rel=1e-12)


def test_layout_and_count():
    # width 32, 4 levels: the widths and concatenations of the documented network
    t = unet.layer_table(32, 4)
    assert [(c, o) for c, o, *_ in t] == [(8, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128), (128, 256),
                                          (256, 256), (384, 128), (128, 128), (192, 64), (64, 64), (96, 32), (32, 32)]
    n = sum(o * ((9 * c + 31) // 32 * 32 + 1) for c, o, *_ in t) + 33
    p = np.zeros(n)
    convs, head = unet.unpack(p, 32, 4)
    assert len(convs) == 14 and head[0].shape == (32,)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -3.14159, 0.0])
    r = unet.bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0  # tie to even
    assert r[2] == 1.0 + 2.0 ** -6     # tie to even (odd neighbour below)
    assert abs(r[3] + 3.14159) <= 2.0 ** -8 * 4 and r[4] == 0.0


@pytest.mark.parametrize("levels", [2, 3])
def test_gradient_by_finite_differences(levels):
    width, n = 8, 8
    p = _params(width, levels, seed=levels)
    rng = np.random.default_rng(10 + levels)
    dh = rng.normal(size=(2, n, n))
    low = rng.normal(size=(2, n, n))
    target = np.abs(rng.normal(size=(2, n, n)))
    loss, g = unet.loss_grad(p, dh, low, target, width, levels)
    assert loss > 0
    idx = np.concatenate([rng.choice(p.size - width - 1, 40, replace=False), np.arange(p.size - width - 1, p.size)])
    eps = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += eps
        lp = unet.loss_grad(q, dh, low, target, width, levels)[0]
        q[i] -= 2 * eps
        lm = unet.loss_grad(q, dh, low, target, width, levels)[0]
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-4 * np.abs(g).max(), i
