"""Pins of the energy and force oracle (Section 3.3 energy expression and
forces; Appendix B overlap correction) for the Gaussian stand-in
pseudocharges: the forces are minus the derivative of the energy with
respect to the atom positions (central differences, phi re-solved), the
overlap correction of an isolated pair is its closed form, the Gaussian
potential solves its Poisson equation."""
import dataclasses
import math

import numpy as np
import pytest
from scipy.special import erfc

from oracle import energy, fd
from paper_1412_8250_amd import inputs

SIGMA, CUT = 0.8, 8.5 * 0.8


def _r_dependent_energy(u, cell, atoms):
    c = dataclasses.replace(cell, atoms=atoms)
    b = inputs.pseudocharge(c, SIGMA)
    e, phi = energy.energy_terms(u, b, c.h, 0.2, atoms, -3.0, SIGMA, CUT)
    return e["electrostatic"] + e["self"] + e["overlap"], phi


def test_forces_are_minus_the_energy_gradient():
    w = inputs.small_cell()
    cell = w.cell
    atoms = np.array(cell.atoms, dtype=float) + np.array([[0.3, -0.2, 0.1], [0.0, 0.25, -0.15],
                                                          [-0.1, 0.0, 0.2], [0.2, 0.1, 0.0]])
    u = np.sqrt(w.rho)
    e0, phi = _r_dependent_energy(u, cell, atoms)
    f = energy.forces(phi, atoms, -3.0, SIGMA, cell.h, CUT)
    d = 1e-4
    for J in (0, 2):
        for a in range(3):
            ap, am = atoms.copy(), atoms.copy()
            ap[J, a] += d
            am[J, a] -= d
            g = (_r_dependent_energy(u, cell, ap)[0] - _r_dependent_energy(u, cell, am)[0]) / (2 * d)
            assert abs(-g - f[J, a]) <= 1e-6 * np.abs(f).max() + 1e-9, (J, a, -g, f[J, a])


def test_overlap_of_an_isolated_pair():
    box = (60.0, 60.0, 60.0)
    for dist in (1.0, 2.5, 4.0):
        atoms = np.array([[10.0, 10.0, 10.0], [10.0 + dist, 10.0, 10.0]])
        e, f = energy.overlap(atoms, -3.0, SIGMA, box)
        assert abs(e - 9.0 * erfc(dist / (2 * SIGMA)) / dist) <= 1e-14 * max(1.0, e)
        # Newton's third law, and the force pushes the pair apart
        assert np.abs(f[0] + f[1]).max() <= 1e-14 and f[1, 0] > 0


def test_gaussian_potential_solves_poisson():
    """-L_h V / (4 pi) = b for the radial pair used in the self and force sums
    (a single Gaussian in a box large enough that images do not matter; the
    12th-order stencil is accurate to ~1e-9 at this resolution away from r = 0)."""
    n, hh = 64, 0.15
    h = (hh,) * 3
    c = n * hh / 2
    z, y, x = np.meshgrid(*(np.arange(n) * hh,) * 3, indexing="ij")
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    v = energy.gauss_v(r, 1.0, 1.0)
    b = energy.gauss_b(r, 1.0, 1.0)
    lap = fd.laplacian(v, h)
    core = r < 2.5
    assert np.abs(-lap[core] / (4 * math.pi) - b[core]).max() <= 1e-6 * b.max()
