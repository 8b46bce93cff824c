"""Pins of the network oracle (learned solver aid): conv against its plain
definition written as explicit loops, FP64 central finite differences of the
loss, positive homogeneity and translation equivariance."""
import numpy as np
import pytest

from oracle import nn


def test_conv_matches_explicit_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(4, 5, 6, 3))
    W = rng.normal(size=(27, 3, 2))
    out = nn.conv(x, W)
    ref = np.zeros((4, 5, 6, 2))
    for z in range(4):
        for y in range(5):
            for xx in range(6):
                for t, (dz, dy, dx) in enumerate(nn.TAPS):
                    ref[z, y, xx] += x[(z + dz) % 4, (y + dy) % 5, (xx + dx) % 6] @ W[t]
    assert np.abs(out - ref).max() < 1e-12


def test_pool_up_shapes_and_adjointness():
    rng = np.random.default_rng(1)
    a = rng.normal(size=(8, 8, 8, 3))
    b = rng.normal(size=(4, 4, 4, 3))
    # <pool(a), b> = <a, pool_grad(b)>  and  <up(b), a> = <b, up_grad(a)>
    assert abs((nn.pool(a) * b).sum() - (a * nn.pool_grad(b)).sum()) < 1e-12
    assert abs((nn.up(b) * a).sum() - (b * nn.up_grad(a)).sum()) < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_gradients_against_central_differences(seed):
    rng = np.random.default_rng(seed)
    W = nn.init_weights(rng)
    g = rng.normal(size=(8, 8, 8))
    target = rng.normal(size=(8, 8, 8))
    out, cache = nn.forward(W, g)
    L, dout = nn.loss(out, target)
    grads = nn.backward(W, cache, dout)
    eps = 1e-6
    for name, ci, co in nn.LAYERS:
        for _ in range(3):
            idx = (rng.integers(27), rng.integers(ci), rng.integers(co))
            Wp = {k: v.copy() for k, v in W.items()}
            Wm = {k: v.copy() for k, v in W.items()}
            Wp[name][idx] += eps
            Wm[name][idx] -= eps
            Lp = nn.loss(nn.forward(Wp, g)[0], target)[0]
            Lm = nn.loss(nn.forward(Wm, g)[0], target)[0]
            num = (Lp - Lm) / (2 * eps)
            ana = grads[name][idx]
            assert abs(num - ana) <= 1e-6 * max(1e-3, abs(ana)) + 1e-9, (name, idx, num, ana)


def test_positive_homogeneity_and_translation_equivariance():
    rng = np.random.default_rng(2)
    W = nn.init_weights(rng)
    g = rng.normal(size=(16, 16, 16))
    out = nn.forward(W, g)[0]
    assert np.abs(nn.forward(W, 3.7 * g)[0] - 3.7 * out).max() < 1e-10 * np.abs(out).max()
    sh = np.roll(g, (8, 0, 8), (0, 1, 2))
    assert np.abs(nn.forward(W, sh)[0] - np.roll(out, (8, 0, 8), (0, 1, 2))).max() < 1e-10 * np.abs(out).max()
