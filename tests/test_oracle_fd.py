"""Pins of the oracle's finite-difference Laplacian (Section 4, FD Laplacian).

Independent facts used: the Taylor (moment) conditions that define a 2N-th
order central second difference, the textbook 2nd/4th/6th-order stencils,
the eigen-structure of a periodic circulant operator (dense eigensolver), and
the convergence order on a smooth periodic function.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import fd


def moment_weights(N):
    """Weights c_0, c_1..c_N of c_0 f(0) + sum_p c_p (f(p) + f(-p)) that reproduce
    f''(0) exactly for all polynomials of degree <= 2N+1 (h = 1)."""
    A = [[Fraction(0)] * (N + 1) for _ in range(N + 1)]
    rhs = [Fraction(0)] * (N + 1)
    for k in range(N + 1):          # monomial x^{2k}
        A[k][0] = Fraction(1 if k == 0 else 0)
        for p in range(1, N + 1):
            A[k][p] = Fraction(2 * p ** (2 * k))
        rhs[k] = Fraction(2 if k == 1 else 0)
    # Gaussian elimination in exact arithmetic
    n = N + 1
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        rhs[c], rhs[piv] = rhs[piv], rhs[c]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c] / A[c][c]
                A[r] = [a - f * b for a, b in zip(A[r], A[c])]
                rhs[r] -= f * rhs[c]
    return [rhs[i] / A[i][i] for i in range(n)]


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_weights_satisfy_moment_conditions(N):
    c = moment_weights(N)
    w = fd.weights_exact(N)
    assert 2 * w[0] == c[0]                 # centre of one axis is 2 w_0
    assert w[1:] == c[1:]


def test_weights_textbook_stencils():
    assert fd.weights_exact(1) == [-1, 1]
    assert fd.weights_exact(2) == [Fraction(-5, 4), Fraction(4, 3), Fraction(-1, 12)]
    assert fd.weights_exact(3) == [Fraction(-49, 36), Fraction(3, 2), Fraction(-3, 20),
                                   Fraction(1, 90)]


def test_weights_twelfth_order_values():
    assert fd.weights_exact(6) == [Fraction(-5369, 3600), Fraction(12, 7), Fraction(-15, 56),
                                   Fraction(10, 189), Fraction(-1, 112), Fraction(2, 1925),
                                   Fraction(-1, 16632)]


@pytest.mark.parametrize("N", [1, 3, 6])
@pytest.mark.parametrize("h", [1.0, 0.375, 0.46875])
def test_c_weights_equal_exact(N, h):
    w = fd.weights(N, h)
    ex = np.array([float(x) for x in fd.weights_exact(N)]) / (h * h)
    assert np.allclose(w, ex, rtol=1e-15, atol=0)
    assert abs(2 * w[0] + 2 * w[1:].sum()) < 1e-13 / (h * h)     # rows sum to zero


@pytest.mark.parametrize("shape,h", [((8, 8, 8), (0.5, 0.5, 0.5)),
                                     ((13, 13, 13), (0.4, 0.4, 0.4)),
                                     ((10, 12, 16), (0.3, 0.45, 0.5))])
def test_plane_waves_are_eigenvectors(shape, h):
    """L_h cos(2 pi k.x/L) = lambda(k) cos(...) for every sampled k."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rng = np.random.default_rng(0)
    lam = fd.symbol(shape, h[::-1][::-1], 6)
    for _ in range(12):
        kz, ky, kx = rng.integers(0, nz), rng.integers(0, ny), rng.integers(0, nx)
        ph = 2 * np.pi * (kx * x / nx + ky * y / ny + kz * z / nz)
        for wave in (np.cos(ph), np.sin(ph)):
            out = fd.laplacian(wave, h, 6)
            assert np.abs(out - lam[kz, ky, kx] * wave).max() <= 1e-13 * np.abs(lam).max()


@pytest.mark.parametrize("shape,N", [((5, 5, 5), 6), ((7, 6, 5), 6), ((6, 6, 6), 3),
                                     ((4, 9, 5), 2)])
def test_dense_operator_is_symmetric_circulant_with_symbol_spectrum(shape, N):
    """Covers grids smaller than the stencil (n < 2N+1): repeated periodic wrapping."""
    h = (0.31, 0.42, 0.53)
    n = int(np.prod(shape))
    M = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        M[:, c] = fd.laplacian(e.reshape(shape), h, N).ravel()
    assert np.abs(M - M.T).max() < 1e-12
    assert np.abs(M.sum(1)).max() < 1e-11          # constants are in the null space
    ev = np.sort(np.linalg.eigvalsh(M))
    sym = np.sort(fd.symbol(shape, h, N).ravel())
    assert np.abs(ev - sym).max() < 1e-11 * np.abs(sym).max()
    # circulant: shifting the input shifts the output
    rng = np.random.default_rng(1)
    v = rng.normal(size=shape)
    a = fd.laplacian(np.roll(v, (1, 2, 3), (0, 1, 2)), h, N)
    b = np.roll(fd.laplacian(v, h, N), (1, 2, 3), (0, 1, 2))
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()


def test_symbol_closed_form_properties():
    th = np.array([0.5, 1.0])
    # 1D symbol of the 12th order stencil against -theta^2 (h = 1)
    w = [float(x) for x in fd.weights_exact(6)]
    s = 2 * w[0] + 2 * sum(w[p] * np.cos(p * th) for p in range(1, 7))
    rel = np.abs(s + th ** 2) / th ** 2
    assert 2.0e-9 < rel[0] < 3.2e-9
    assert 7.0e-6 < rel[1] < 9.5e-6
    smax = 2 * w[0] + 2 * sum(w[p] * np.cos(p * np.pi) for p in range(1, 7))
    assert abs(smax + 7.072939) < 1e-6
    lam = fd.symbol((16, 16, 16), (0.5,) * 3, 6)
    assert lam[0, 0, 0] == 0.0 or abs(lam[0, 0, 0]) < 1e-12
    assert (lam.ravel()[1:] < 0).all()


@pytest.mark.parametrize("N,ns,order", [(1, (16, 32), 2), (2, (16, 32), 4), (3, (16, 24), 6),
                                        (6, (32, 40), 12)])
def test_convergence_order_on_smooth_function(N, ns, order):
    """Error of L_h f against the exact Laplacian decays like h^(2N)."""
    L = 2 * np.pi
    errs = []
    for n in ns:
        h = L / n
        xs = np.arange(n) * h
        f1 = np.exp(0.3 * np.sin(xs))
        d2 = f1 * (0.09 * np.cos(xs) ** 2 - 0.3 * np.sin(xs))
        f = np.broadcast_to(f1[None, None, :], (4, 4, n)).copy()
        out = fd.laplacian(f, (h, 1.0, 1.0), N)[0, 0]
        errs.append(np.abs(out - d2).max())
    slope = np.log(errs[0] / errs[1]) / np.log(ns[1] / ns[0])
    assert order - 0.7 < slope < order + 1.5, (errs, slope)


def test_laplacian_at_matches_full_apply():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(9, 11, 14))
    h = (0.3, 0.4, 0.5)
    full = fd.laplacian(x, h, 6)
    pts = [(0, 0, 0), (8, 10, 13), (4, 5, 6), (1, 9, 12)]
    assert np.allclose(fd.laplacian_at(x, h, 6, pts), [full[p] for p in pts], rtol=1e-14, atol=1e-12)


def test_complex_apply_acts_on_parts():
    rng = np.random.default_rng(4)
    a, b = rng.normal(size=(2, 8, 9, 10))
    h = (0.3, 0.4, 0.5)
    out = fd.laplacian(a + 1j * b, h, 6)
    assert np.allclose(out, fd.laplacian(a, h, 6) + 1j * fd.laplacian(b, h, 6), rtol=0, atol=1e-13)
