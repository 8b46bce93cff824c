"""Pins of the density update U(v) (Appendix C, Algorithm 1; Section 3.3 Euler-Lagrange)."""
import numpy as np

from oracle import density, poisson, xc
from paper_1412_8250_amd import inputs


def _cell():
    w = inputs.small_cell()
    g, _ = poisson.rhs(w.rho, w.b)
    return w, poisson.solve_exact(g, w.cell.h)


def test_lambda_zero_matches_pointwise_brute_force():
    w, phi = _cell()
    u, it, res, eta = density.update(np.sqrt(w.rho), phi, w.cell.h, 0.0, w.cell.n_electrons,
                                     tol=1e-10)
    up, etap = density.pointwise_minimiser(phi, w.cell.h, w.cell.n_electrons)
    assert res <= 1e-10
    assert abs(eta - etap) < 1e-9
    assert np.abs(u - up).max() < 1e-7 * np.abs(up).max()


def test_uniform_potential_gives_uniform_density():
    w, _ = _cell()
    v = np.full(w.cell.shape, 0.37)
    u, it, res, eta = density.update(np.sqrt(w.rho), v, w.cell.h, 0.2, w.cell.n_electrons)
    ubar = np.sqrt(w.cell.n_electrons / w.cell.volume)
    assert np.abs(u - ubar).max() < 1e-9 * ubar
    rho = ubar ** 2
    assert abs(eta - (xc.v_tf(rho) + xc.v_xc(rho) + 0.37)) < 1e-9


def test_tfw_update_solves_euler_lagrange_and_keeps_constraint():
    w, phi = _cell()
    u, it, res, eta = density.update(np.sqrt(w.rho), phi, w.cell.h, 0.2, w.cell.n_electrons)
    dv = np.prod(w.cell.h)
    assert abs(dv * (u * u).sum() - w.cell.n_electrons) < 1e-11 * w.cell.n_electrons
    r, eta2 = density.el_residual(u, phi, w.cell.h, 0.2, w.cell.n_electrons)
    assert r <= 1e-10 and abs(eta - eta2) < 1e-12
    assert (u > 0).all()
    # the result is a minimum on the constraint sphere: random feasible perturbations raise E
    rng = np.random.default_rng(5)
    e0 = density.energy(u, phi, w.cell.h, 0.2)
    for _ in range(3):
        p = u + 1e-4 * rng.normal(size=u.shape) * u
        p *= np.sqrt(w.cell.n_electrons / (dv * (p * p).sum()))
        assert density.energy(p, phi, w.cell.h, 0.2) > e0


def test_gradient_of_energy_is_twice_hamiltonian():
    w, phi = _cell()
    rng = np.random.default_rng(6)
    u = np.sqrt(w.rho)
    d = rng.normal(size=u.shape) * u
    dv = np.prod(w.cell.h)
    eps = 1e-6
    num = (density.energy(u + eps * d, phi, w.cell.h, 0.2) -
           density.energy(u - eps * d, phi, w.cell.h, 0.2)) / (2 * eps)
    ana = 2 * dv * (density.hamiltonian(u, phi, w.cell.h, 0.2) * d).sum()
    assert abs(num - ana) < 1e-7 * abs(ana)
