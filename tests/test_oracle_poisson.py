"""Pins of the oracle's periodic Poisson solve (Section 3.3 Poisson equation;
Section 4 zero-integral convention).

Independent facts: the continuum periodic potential of Gaussian charges has a
closed-form Fourier series, and the discrete solution must converge to it at
the stencil's order; two unrelated discrete routes (DFT diagonalisation and
textbook CG) must agree; a uniform neutral system has zero potential.
"""
import numpy as np
import pytest

from oracle import fd, poisson
from paper_1412_8250_amd import inputs

L = 7.5
CENTRES = np.array([[1.0, 2.0, 3.0], [4.5, 5.0, 1.5]])
CHARGES = np.array([1.0, -1.0])


def gaussians_on_grid(n, sigma):
    h = L / n
    x = np.arange(n) * h
    b = np.zeros((n, n, n))
    for r, qq in zip(CENTRES, CHARGES):
        fs = []
        for a in range(3):
            d = (x - r[a])[:, None] + L * np.arange(-3, 4)[None, :]
            fs.append(np.exp(-d ** 2 / (2 * sigma ** 2)).sum(1))
        b += qq * (2 * np.pi * sigma ** 2) ** -1.5 * fs[2][:, None, None] * fs[1][None, :, None] * fs[0][None, None, :]
    return b


def continuum_potential(n, sigma, K=40):
    """phi(x) = (4 pi / Omega) sum_{G != 0} sum_J q_J exp(-sigma^2 G^2 / 2) exp(iG.(x-R_J)) / G^2
    sampled at the grid points (the Fourier series is folded onto the grid's DFT)."""
    m = np.arange(-K, K + 1)
    G = 2 * np.pi * m / L
    GZ, GY, GX = np.meshgrid(G, G, G, indexing="ij")
    MZ, MY, MX = np.meshgrid(m, m, m, indexing="ij")
    G2 = GX ** 2 + GY ** 2 + GZ ** 2
    S = np.zeros(G2.shape, complex)
    for r, qq in zip(CENTRES, CHARGES):
        S += qq * np.exp(-1j * (GX * r[0] + GY * r[1] + GZ * r[2]))
    coef = np.where(G2 == 0, 0, 4 * np.pi / L ** 3 * S * np.exp(-sigma ** 2 * G2 / 2) /
                    np.where(G2 == 0, 1, G2))
    c = np.zeros((n, n, n), complex)
    np.add.at(c, (MZ % n, MY % n, MX % n), coef)
    return np.real(np.fft.ifftn(c)) * n ** 3


def test_converges_to_continuum_gaussian_potential_at_twelfth_order():
    errs = []
    ns = (32, 40)
    for n in ns:
        b = gaussians_on_grid(n, 1.2)
        g, _ = poisson.rhs(np.zeros_like(b), b)
        ph = poisson.solve_exact(g, (L / n,) * 3)
        ex = continuum_potential(n, 1.2)
        errs.append(np.abs(ph - ex).max() / np.abs(ex).max())
    slope = np.log(errs[0] / errs[1]) / np.log(ns[1] / ns[0])
    assert 11.0 < slope < 13.5, (errs, slope)
    assert errs[1] < 2e-11


def test_small_cell_potential_close_to_continuum():
    """At the 16^3 small-cell resolution (sigma = 0.8) the discrete potential is
    within the expected discretisation error of the analytic one."""
    b = gaussians_on_grid(16, 0.8)
    g, _ = poisson.rhs(np.zeros_like(b), b)
    ph = poisson.solve_exact(g, (L / 16,) * 3)
    err = np.abs(ph - continuum_potential(16, 0.8)).max() / np.abs(ph).max()
    assert 1e-6 < err < 5e-5


@pytest.mark.parametrize("shape,h", [((8, 8, 8), (0.5,) * 3), ((9, 10, 12), (0.4, 0.45, 0.5)),
                                     ((16, 16, 16), (0.46875,) * 3)])
def test_spectral_and_cg_agree(shape, h):
    rng = np.random.default_rng(7)
    g = rng.normal(size=shape)
    g -= g.mean()
    a = poisson.solve_exact(g, h)
    b, it, rel = poisson.solve_cg(g, h, tol=1e-13)
    assert rel < 1e-12
    assert np.abs(a - b).max() <= 1e-10 * np.abs(a).max()
    assert abs(a.sum()) < 1e-10 * np.abs(a).sum() and abs(b.sum()) < 1e-10 * np.abs(b).sum()
    assert poisson.residual(a, g, h) < 1e-13


def test_small_cell_workload():
    w = inputs.small_cell()
    g, removed = poisson.rhs(w.rho, w.b)
    assert abs(removed) < 1e-12                 # generator makes the cell neutral
    phi = poisson.solve_exact(g, w.cell.h)
    x, it, rel = poisson.solve_cg(g, w.cell.h, tol=1e-10)
    assert rel <= 1e-10
    assert np.abs(phi - x).max() < 1e-9 * np.abs(phi).max()


def test_uniform_neutral_system_has_zero_potential():
    j = inputs.jellium(1, 12)
    g, _ = poisson.rhs(j.rho, j.b)
    assert np.abs(poisson.solve_exact(g, j.cell.h)).max() < 1e-13


def test_non_neutral_rhs_is_projected():
    rng = np.random.default_rng(8)
    rho = rng.uniform(0.01, 0.02, size=(10, 10, 10))
    b = np.full_like(rho, -0.001)
    g, removed = poisson.rhs(rho, b)
    assert abs(removed - 4 * np.pi * (rho + b).mean()) < 1e-15
    assert abs(g.mean()) < 1e-15
