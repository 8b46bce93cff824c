"""Finite-difference Laplacian and gradient of order 2N on a periodic uniform
grid.

Section 4, FD Laplacian equation: the Laplacian at (i,j,k) is the sum over
p = 0..N of w_p times the six values at offsets +-p along each axis, with the
weight formulas given there; indices outside the grid map to their periodic
images.  Section 4, FD gradient equation: each component is the sum over
p = 1..N of w~_p times the difference of the values at offsets +p and -p
along its axis.
"""
from fractions import Fraction
from math import factorial

import numpy as np

from ._clib import lib, ptr


def weights_exact(N: int):
    """Exact rational weights for h = 1 (w_0, w_1, ..., w_N)."""
    w0 = -sum(Fraction(1, q * q) for q in range(1, N + 1))
    ws = [w0]
    for p in range(1, N + 1):
        ws.append(Fraction(2 * (-1) ** (p + 1) * factorial(N) ** 2,
                           p * p * factorial(N - p) * factorial(N + p)))
    return ws


def gradient_weights_exact(N: int):
    """Exact rational first-derivative weights w~_1 .. w~_N for h = 1
    (Section 4, the weights of the FD gradient equation)."""
    return [Fraction((-1) ** (p + 1) * factorial(N) ** 2, p * factorial(N - p) * factorial(N + p))
            for p in range(1, N + 1)]


def gradient(x: np.ndarray, h_xyz, N: int = 6):
    """(d/dx, d/dy, d/dz) of a real [nz][ny][nx] array by the periodic FD
    gradient: sum_p w~_p / h (f(i + p) - f(i - p)) along each axis."""
    x = np.asarray(x, dtype=np.float64)
    out = []
    for axis, hh in zip((2, 1, 0), h_xyz):
        w = [float(c) / hh for c in gradient_weights_exact(N)]
        g = np.zeros_like(x)
        for p in range(1, N + 1):
            g += w[p - 1] * (np.roll(x, -p, axis=axis) - np.roll(x, p, axis=axis))
        out.append(g)
    return tuple(out)


def weights(N: int, h: float) -> np.ndarray:
    """FP64 weights for spacing h, from the C oracle."""
    w = np.zeros(N + 1)
    lib().orc_fd_weights(N, float(h), ptr(w))
    return w


def symbol_1d(n: int, h: float, N: int) -> np.ndarray:
    """Eigenvalues of the 1D periodic stencil on exp(i 2 pi k j / n), k = 0..n-1:
    2 w_0 + 2 sum_p w_p cos(p theta_k), theta_k = 2 pi k / n."""
    w = [float(x) / (h * h) for x in weights_exact(N)]
    theta = 2.0 * np.pi * np.arange(n) / n
    return 2.0 * w[0] + 2.0 * sum(w[p] * np.cos(p * theta) for p in range(1, N + 1))


def symbol(shape_zyx, h_xyz, N: int) -> np.ndarray:
    """Eigenvalue lambda(k) of L_h for every FFT frequency, array [kz][ky][kx]."""
    nz, ny, nx = shape_zyx
    hx, hy, hz = h_xyz
    lx, ly, lz = symbol_1d(nx, hx, N), symbol_1d(ny, hy, N), symbol_1d(nz, hz, N)
    return lz[:, None, None] + ly[None, :, None] + lx[None, None, :]


def _dims(x, h_xyz):
    nz, ny, nx = x.shape
    hx, hy, hz = h_xyz
    return nx, ny, nz, float(hx), float(hy), float(hz)


def laplacian(x: np.ndarray, h_xyz, N: int = 6) -> np.ndarray:
    """L_h x for a real or complex [nz][ny][nx] array."""
    if np.iscomplexobj(x):
        xc = np.ascontiguousarray(x, dtype=np.complex128)
        y = np.empty_like(xc)
        lib().orc_laplacian_z(*_dims(xc, h_xyz), N, ptr(xc), ptr(y))
        return y
    xr = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(xr)
    lib().orc_laplacian(*_dims(xr, h_xyz), N, ptr(xr), ptr(y))
    return y


def laplacian_at(x: np.ndarray, h_xyz, N: int, points) -> np.ndarray:
    """L_h x at selected points (k, j, i) only, straight from the definition."""
    nz, ny, nx = x.shape
    wx, wy, wz = (weights(N, h) for h in h_xyz)
    out = []
    for (k, j, i) in points:
        s = 2.0 * (wx[0] + wy[0] + wz[0]) * x[k, j, i]
        for p in range(1, N + 1):
            s += wx[p] * (x[k, j, (i + p) % nx] + x[k, j, (i - p) % nx])
            s += wy[p] * (x[k, (j + p) % ny, i] + x[k, (j - p) % ny, i])
            s += wz[p] * (x[(k + p) % nz, j, i] + x[(k - p) % nz, j, i])
        out.append(s)
    return np.array(out)


def threads() -> int:
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """OpenMP threads of later oracle calls (timing on one core or all)."""
    lib().orc_set_threads(int(n))
