"""Pins of the oracle's complex shifted solve (Section 3.1, Helmholtz equations;
Appendix A shift table and conjugate-pair rule)."""
import numpy as np
import pytest

from oracle import fd, helmholtz, kernel
from paper_1412_8250_amd import inputs


@pytest.mark.parametrize("kappa", [0.1 + 0.0j, 2.0 + 1.5j, 5.0 * np.exp(0.45j * np.pi),
                                   -1.680 - 1.660j, 0.236 - 0.926j])
def test_spectral_and_cocg_agree(kappa):
    rng = np.random.default_rng(11)
    shape, h = (10, 9, 12), (0.42, 0.47, 0.39)
    f = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    a = helmholtz.solve_exact(f, kappa, h)
    b, it, rel = helmholtz.solve_cocg(f, kappa, h, tol=1e-13)
    assert it > 0 and rel < 1e-12
    assert np.abs(a - b).max() <= 1e-10 * np.abs(a).max()
    assert helmholtz.residual(a, f, kappa, h) < 1e-13


def test_single_plane_wave_closed_form():
    """A plane wave is an eigenvector: u = f / (-lambda(k) + kappa) with the 1D
    symbols of Section 4's weights written out here for this wave."""
    n, h = 12, 0.5
    k = (2, 5, 1)          # (kx, ky, kz)
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    f = np.exp(2j * np.pi * (k[0] * x + k[1] * y + k[2] * z) / n)
    w = [float(c) / h ** 2 for c in fd.weights_exact(6)]
    lam = sum(2 * w[0] + 2 * sum(w[p] * np.cos(2 * np.pi * p * kk / n) for p in range(1, 7)) for kk in k)
    kappa = 0.7 - 0.3j
    u = helmholtz.solve_exact(f, kappa, (h,) * 3)
    assert np.abs(u - f / (-lam + kappa)).max() < 1e-13


def test_conjugate_pair_invariant():
    rng = np.random.default_rng(12)
    f = rng.normal(size=(8, 8, 8)) + 1j * rng.normal(size=(8, 8, 8))
    h = (0.5,) * 3
    k = 0.3 + 1.1j
    u1 = helmholtz.solve_exact(f, k, h)
    u2 = helmholtz.solve_exact(np.conj(f), np.conj(k), h)
    assert np.abs(u2 - np.conj(u1)).max() < 1e-13


def test_paper_shift_table_and_fermi_wavevector():
    # Al at a = 7.5 bohr: rho_bar = 12 / 7.5^3
    kf = kernel.fermi_wavevector(12.0, 7.5 ** 3)
    assert abs(kf - 0.94436) < 5e-5
    ks = kernel.shifts(12.0, 7.5 ** 3)
    assert abs(ks[0] - (-1.680 - 1.660j)) < 2e-3
    assert abs(ks[2] - (0.236 - 0.926j)) < 2e-3
    assert ks[1] == np.conj(ks[0]) and ks[3] == np.conj(ks[2])
    assert np.all(ks[4:] == ks[:4])
    assert kernel.P00[1] == np.conj(kernel.P00[0]) and kernel.P00[3] == np.conj(kernel.P00[2])


def test_kernel_potential_is_real_and_vanishes_for_uniform_density():
    w = inputs.small_cell()
    V = kernel.solve_all(w.rho, w.cell.h, w.cell.n_electrons, w.cell.volume)
    # conjugate pairs: V_2 = conj(V_1), V_4 = conj(V_3) for a real density
    assert np.abs(V[1] - np.conj(V[0])).max() < 1e-13 * np.abs(V[0]).max()
    assert np.abs(V[3] - np.conj(V[2])).max() < 1e-13 * np.abs(V[2]).max()
    j = inputs.jellium(1, 16)
    Vj = kernel.solve_all(j.rho, j.cell.h, j.cell.n_electrons, j.cell.volume)
    assert max(np.abs(v).max() for v in Vj) < 1e-12
