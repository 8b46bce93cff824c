"""FP64 reference of the learned solver aid's network (test infrastructure).

The paper has no network; its conclusion calls for real-space preconditioners
(multigrid) to make iteration counts size-independent (Section 5.5).  The
network here approximates the inverse of the dimensionless operator -h^2 L_h on
a periodic grid.  Architecture (channels-last arrays [z][y][x][C]):

  level 0 (n):    c0a 1->16,  c0b 16->16                      -> skip s0
  level 1 (n/2):  pool, c1a 16->32, c1b 32->32                -> skip s1
  level 2 (n/4):  pool, c2a 32->64, c2b 64->64                -> skip s2
  level 3 (n/8):  pool, c3a 64->64, c3b 64->64
  up, concat s2 (128): d2a 128->64, d2b 64->64
  up, concat s1 (96):  d1a 96->32,  d1b 32->32
  up, concat s0 (48):  d0a 48->16,  d0b 16->16
  out 16->1 (no activation)

Every conv is 3x3x3 with periodic padding, bias-free, followed by ReLU except
the last.  Pool = 2x2x2 average; up = nearest-neighbour 2x; concat order is
[upsampled, skip].  Without biases, ReLU, average pooling and nearest
upsampling are all positively homogeneous, so N(c x) = c N(x) for c > 0.
Weights are stored W[t][ci][co] with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1).
"""
import numpy as np

LAYERS = [  # name, cin, cout
    ("c0a", 1, 16), ("c0b", 16, 16),
    ("c1a", 16, 32), ("c1b", 32, 32),
    ("c2a", 32, 64), ("c2b", 64, 64),
    ("c3a", 64, 64), ("c3b", 64, 64),
    ("d2a", 128, 64), ("d2b", 64, 64),
    ("d1a", 96, 32), ("d1b", 32, 32),
    ("d0a", 48, 16), ("d0b", 16, 16),
    ("out", 16, 1),
]
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def init_weights(rng: np.random.Generator):
    """He-normal initialisation (fan-in 27 cin)."""
    return {name: rng.normal(0.0, np.sqrt(2.0 / (27 * ci)), size=(27, ci, co))
            for name, ci, co in LAYERS}


def shift(x, dz, dy, dx):
    """y[z, y, x] = x[z + dz, y + dy, x + dx] with periodic wrap."""
    return np.roll(x, (-dz, -dy, -dx), axis=(0, 1, 2))


def conv(x, W):
    """out[p, co] = sum_t sum_ci x[p + off_t, ci] W[t, ci, co]."""
    out = np.zeros(x.shape[:3] + (W.shape[2],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        out += shift(x, dz, dy, dx) @ W[t]
    return out


def conv_grad(x, W, dy):
    """Gradients of conv w.r.t. its input and weights given dL/d(out)."""
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for t, (a, b, c) in enumerate(TAPS):
        xs = shift(x, a, b, c)
        dW[t] = np.einsum("zyxi,zyxo->io", xs, dy)
        dx += shift(dy @ W[t].T, -a, -b, -c)
    return dx, dW


def pool(x):
    n0, n1, n2, c = x.shape
    return x.reshape(n0 // 2, 2, n1 // 2, 2, n2 // 2, 2, c).mean(axis=(1, 3, 5))


def pool_grad(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, 0), 2, 1), 2, 2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up_grad(dy):
    n0, n1, n2, c = dy.shape
    return dy.reshape(n0 // 2, 2, n1 // 2, 2, n2 // 2, 2, c).sum(axis=(1, 3, 5))


def relu(x):
    return np.maximum(x, 0.0)


def forward(W, g):
    """g: [n][n][n] -> (output [n][n][n], cache of activations)."""
    cache = {}
    x = g[..., None]

    def cr(name, x):
        cache[name + ".in"] = x
        y = conv(x, W[name])
        cache[name + ".pre"] = y
        return relu(y)

    s0 = cr("c0b", cr("c0a", x))
    s1 = cr("c1b", cr("c1a", pool(s0)))
    s2 = cr("c2b", cr("c2a", pool(s1)))
    b = cr("c3b", cr("c3a", pool(s2)))
    d2 = cr("d2b", cr("d2a", np.concatenate([up(b), s2], -1)))
    d1 = cr("d1b", cr("d1a", np.concatenate([up(d2), s1], -1)))
    d0 = cr("d0b", cr("d0a", np.concatenate([up(d1), s0], -1)))
    cache["out.in"] = d0
    out = conv(d0, W["out"])
    return out[..., 0], cache


def backward(W, cache, dout):
    """dL/dW for every layer given dL/d(output) ([n][n][n])."""
    grads = {}

    def back(name, dy_post):
        dy = dy_post * (cache[name + ".pre"] > 0)
        dx, grads[name] = conv_grad(cache[name + ".in"], W[name], dy)
        return dx

    dx, grads["out"] = conv_grad(cache["out.in"], W["out"], dout[..., None])
    dx = back("d0a", back("d0b", dx))
    c1 = cache["d1b.pre"].shape[-1]       # channels of the upsampled branch at level 0 = 32
    d_up1, d_s0 = dx[..., :c1], dx[..., c1:]
    dx = back("d1a", back("d1b", up_grad(d_up1)))
    c2 = cache["d2b.pre"].shape[-1]       # 64
    d_up2, d_s1 = dx[..., :c2], dx[..., c2:]
    dx = back("d2a", back("d2b", up_grad(d_up2)))
    c3 = cache["c3b.pre"].shape[-1]       # 64
    d_up3, d_s2 = dx[..., :c3], dx[..., c3:]
    dx = back("c3a", back("c3b", up_grad(d_up3)))
    dx = back("c2a", back("c2b", pool_grad(dx) + d_s2))
    dx = back("c1a", back("c1b", pool_grad(dx) + d_s1))
    dx = back("c0a", back("c0b", pool_grad(dx) + d_s0))
    return grads


def loss(out, target):
    """Relative squared error ||out - target||^2 / ||target||^2 and its gradient."""
    den = float((target * target).sum())
    diff = out - target
    return float((diff * diff).sum()) / den, 2.0 * diff / den


def loss_energy(out, target, h):
    """Relative energy-norm error e^T A e / t^T A t, e = out - target, with
    A = -h2 L_h the order-12 FD operator of Section 4 (h2 = (hx hy hz)^(2/3)),
    and its gradient 2 A e / t^T A t (A is symmetric)."""
    from . import fd
    h2 = float(np.cbrt(h[0] * h[1] * h[2])) ** 2

    def A(v):
        return -h2 * fd.laplacian(v, h)

    den = float((target * A(target)).sum())
    e = out - target
    Ae = A(e)
    return float((e * Ae).sum()) / den, 2.0 * Ae / den


def loss_residual(out, target, h):
    """Relative residual-norm error ||A e||^2 / ||A target||^2 (A as in
    loss_energy) and its gradient 2 A A e / ||A target||^2."""
    from . import fd
    h2 = float(np.cbrt(h[0] * h[1] * h[2])) ** 2

    def A(v):
        return -h2 * fd.laplacian(v, h)

    At = A(target)
    den = float((At * At).sum())
    Ae = A(out - target)
    return float((Ae * Ae).sum()) / den, 2.0 * A(Ae) / den
