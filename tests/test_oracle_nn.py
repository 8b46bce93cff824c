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


@pytest.mark.parametrize("power", [1, 2])
def test_operator_loss_spectral_form_and_gradient(power):
    """The energy-norm (power 1) and residual-norm (power 2) losses equal
    their Fourier forms sum lambda^p |e_k|^2 / sum lambda^p |t_k|^2 with the
    exact symbol of -h2 L_h, are unchanged by a constant added to the output
    (constants are the null space), vanish at the target, and their
    gradients match central differences."""
    fn = nn.loss_energy if power == 1 else nn.loss_residual
    from oracle import fd
    rng = np.random.default_rng(3)
    shape, h = (8, 10, 12), (0.4, 0.45, 0.5)
    out = rng.normal(size=shape)
    t = rng.normal(size=shape)
    L, dout = fn(out, t, h)
    h2 = np.cbrt(h[0] * h[1] * h[2]) ** 2
    lam = (-h2 * fd.symbol(shape, h, 6)) ** power
    ek, tk = np.fft.fftn(out - t), np.fft.fftn(t)
    spec = float((lam * abs(ek) ** 2).sum() / (lam * abs(tk) ** 2).sum())
    assert abs(L - spec) <= 1e-12 * spec
    assert abs(fn(out + 3.7, t, h)[0] - L) <= 1e-11 * L
    assert fn(t, t, h)[0] == 0.0
    eps = 1e-6
    for _ in range(5):
        idx = tuple(int(rng.integers(s)) for s in shape)
        op, om = out.copy(), out.copy()
        op[idx] += eps
        om[idx] -= eps
        num = (fn(op, t, h)[0] - fn(om, t, h)[0]) / (2 * eps)
        assert abs(num - dout[idx]) <= 1e-6 * abs(dout[idx]) + 1e-10
