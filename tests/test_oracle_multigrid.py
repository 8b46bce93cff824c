"""Pins of the reference multigrid cycle: dense matrices built point by point
(7-point operator, trilinear prolongation, restriction = P^T / 8, dense
coarsest solve), the exact inverse on one-level grids, symmetry."""
import itertools

import numpy as np
import pytest

from oracle import multigrid as mg


def _dense_A(shape, c, kappa):
    nz, ny, nx = shape
    n = nz * ny * nx
    A = np.zeros((n, n), dtype=complex)
    idx = lambda z, y, x: (z % nz) * ny * nx + (y % ny) * nx + (x % nx)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        i = idx(z, y, x)
        A[i, i] += 2 * sum(c) + kappa
        for (dz, dy, dx), ca in (((0, 0, 1), c[0]), ((0, 1, 0), c[1]), ((1, 0, 0), c[2])):
            A[i, idx(z + dz, y + dy, x + dx)] -= ca
            A[i, idx(z - dz, y - dy, x - dx)] -= ca
    return A


def _dense_P(cshape):
    """Trilinear prolongation from cshape to 2 * cshape, entry by entry."""
    cz, cy, cx = cshape
    fz, fy, fx = 2 * cz, 2 * cy, 2 * cx

    def w1(i, I, nc):       # weight of coarse index I for fine index i on one axis
        if i % 2 == 0:
            return 1.0 if I == i // 2 else 0.0
        return 0.5 if I in (i // 2, (i // 2 + 1) % nc) else 0.0

    P = np.zeros((fz * fy * fx, cz * cy * cx))
    for z, y, x in itertools.product(range(fz), range(fy), range(fx)):
        for Z, Y, X in itertools.product(range(cz), range(cy), range(cx)):
            w = w1(z, Z, cz) * w1(y, Y, cy) * w1(x, X, cx)
            if w:
                P[(z * fy + y) * fx + x, (Z * cy + Y) * cx + X] = w
    return P


def _dense_cycle(f, shape, c, kappa, nu, omega, coarse_max):
    A = _dense_A(shape, c, kappa)
    if max(shape) <= coarse_max:
        return np.linalg.pinv(A) @ f
    d = np.diag(A)
    cshape = tuple(s // 2 for s in shape)
    P = _dense_P(cshape)
    R = P.T / 8.0
    u = np.zeros_like(f)
    for _ in range(nu):
        u = u + omega * (f - A @ u) / d
    uc = _dense_cycle(R @ (f - A @ u), cshape, [ca / 4 for ca in c], kappa, nu, omega, coarse_max)
    u = u + P @ uc
    for _ in range(nu):
        u = u + omega * (f - A @ u) / d
    return u


@pytest.mark.parametrize("kappa", [0.0, 0.7 - 1.3j, -1.6 - 1.6j])
def test_cycle_equals_dense_matrix_construction(kappa):
    """Three levels (8x8x16 -> 4x4x8 -> 2x2x4 with coarse_max 4), anisotropic
    spacings."""
    shape, h = (8, 8, 16), (0.4, 0.5, 0.45)
    c = [1 / v ** 2 for v in h]
    rng = np.random.default_rng(4)
    f = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    if kappa == 0.0:
        f = f.real - f.real.mean()
    got = mg.vcycle(f, h, kappa, coarse_max=4)
    ref = _dense_cycle(f.reshape(-1).astype(complex), shape, c, kappa, 2, 0.8, 4).reshape(shape)
    assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


def test_restriction_is_prolongation_transpose_over_8():
    rng = np.random.default_rng(1)
    a = rng.normal(size=(6, 8, 4))
    b = rng.normal(size=(3, 4, 2))
    assert abs(np.vdot(mg.restrict(a), b) - np.vdot(a, mg.prolong(b)) / 8) <= 1e-12 * np.abs(a).sum()


@pytest.mark.parametrize("kappa", [0.0, 0.3 + 2.0j, -1.6 - 1.6j])
def test_one_level_is_the_exact_inverse(kappa):
    shape, h = (12, 16, 10), (0.5, 0.4, 0.45)
    c = [1 / v ** 2 for v in h]
    rng = np.random.default_rng(2)
    f = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    if kappa == 0.0:
        f = f - f.mean()
    u = mg.vcycle(f, h, kappa)
    assert np.abs(mg.apply7(u, c, kappa) - f).max() <= 1e-11 * np.abs(f).max()
    if kappa == 0.0:
        assert abs(u.mean()) <= 1e-13 * np.abs(u).max()


def test_cycle_is_complex_symmetric_and_positive_for_poisson():
    shape, h = (32, 32, 64), (0.45, 0.4, 0.5)
    rng = np.random.default_rng(3)
    a = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    b = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    k = -1.2 + 0.9j
    x1 = np.sum(mg.vcycle(a, h, k) * b)
    x2 = np.sum(a * mg.vcycle(b, h, k))
    assert abs(x1 - x2) <= 1e-12 * np.abs(a).sum() * np.abs(b).max()
    ar = a.real - a.real.mean()
    assert np.sum(ar * mg.vcycle(ar, h)) > 0
