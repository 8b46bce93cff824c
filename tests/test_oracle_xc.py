"""Pins of the pointwise potentials (Section 2 LDA energy; Section 3.3 potentials)."""
import numpy as np

from oracle import xc


def test_exchange_energy_textbook_value():
    # uniform-gas exchange energy per electron: -0.458165 / r_s hartree
    for r in (0.5, 1.0, 2.0, 4.0):
        rho = 3.0 / (4.0 * np.pi * r ** 3)
        assert abs(xc.eps_x(rho) * r + 0.4581653) < 2e-7


def test_thomas_fermi_constant():
    assert abs(xc.C_F - 2.871234) < 1e-6


def test_potentials_are_density_derivatives():
    """V = d(rho eps)/d rho on both branches of the correlation fit, away from r_s = 1."""
    for rho in (0.002, 0.0284, 0.05, 0.5, 2.0):
        d = 1e-6 * rho
        for e, v in ((lambda r: xc.eps_xc(r) * r, xc.v_xc), (xc.e_tf, xc.v_tf)):
            num = (e(rho + d) - e(rho - d)) / (2 * d)
            assert abs(num - v(rho)) < 1e-7 * max(1.0, abs(v(rho)))


def test_correlation_nearly_continuous_at_rs_one():
    rho1 = 3.0 / (4.0 * np.pi)
    lo, hi = rho1 * (1 + 1e-12), rho1 * (1 - 1e-12)     # r_s just below / above 1
    assert xc.rs(lo) < 1.0 < xc.rs(hi)
    assert abs(xc.eps_c(lo) - xc.eps_c(hi)) < 5e-5
    assert abs(xc.v_c(lo) - xc.v_c(hi)) < 5e-5
