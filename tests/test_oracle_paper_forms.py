"""Pins of the oracle's paper-form pieces: the FD gradient (Section 4, FD
gradient equation), the gradient form of the von Weizsacker energy (Section
3.3 energy expression) and the grid form of the overlap correction with its
extra Poisson solve (Appendix B).

Independent facts used: the Taylor moment conditions of a 2N-th order
central first difference (exact rational arithmetic), the textbook 2nd and
4th order stencils, antisymmetry of a periodic central difference, the
convergence order on a smooth periodic function, the exact gradient energy
of a plane wave, and for Appendix B the closed form of the Gaussians' pair
repulsion (the grid form must converge to E_c(s) - E_c(s_ref) and its forces
to the closed-form forces as h -> 0) plus central differences of the grid
energy itself."""
import dataclasses
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import energy, fd
from paper_1412_8250_amd import inputs


def first_derivative_moment_weights(N):
    """c_1..c_N of sum_p c_p (f(p) - f(-p)) = f'(0) for every polynomial of
    degree <= 2N (h = 1): sum_p 2 p^(2k+1) c_p = [k == 0], k = 0..N-1."""
    A = [[Fraction(2 * p ** (2 * k + 1)) for p in range(1, N + 1)] for k in range(N)]
    rhs = [Fraction(1 if k == 0 else 0) for k in range(N)]
    n = N
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
def test_gradient_weights_satisfy_the_moment_conditions(N):
    assert fd.gradient_weights_exact(N) == first_derivative_moment_weights(N)


def test_gradient_weights_textbook_low_orders():
    assert fd.gradient_weights_exact(1) == [Fraction(1, 2)]
    assert fd.gradient_weights_exact(2) == [Fraction(2, 3), Fraction(-1, 12)]


def test_gradient_is_antisymmetric_and_axis_correct():
    rng = np.random.default_rng(3)
    shape, h = (9, 11, 14), (0.3, 0.4, 0.5)
    f, g = rng.normal(size=(2,) + shape)
    gf, gg = fd.gradient(f, h), fd.gradient(g, h)
    for a in range(3):
        assert abs(np.sum(gf[a] * g) + np.sum(f * gg[a])) <= 1e-12 * np.abs(gf[a]).sum()
    # a function of x alone has no y or z derivative, and vice versa
    x = np.arange(shape[2]) * h[0]
    fx = np.broadcast_to(np.sin(2 * math.pi * x / (shape[2] * h[0])), shape)
    gx, gy, gz = fd.gradient(fx, h)
    assert np.abs(gy).max() == 0 and np.abs(gz).max() == 0 and np.abs(gx).max() > 0.1


@pytest.mark.parametrize("N", [2, 4, 6])
def test_gradient_converges_at_order_2N(N):
    errs = []
    for n in (24, 32):
        L = 2 * math.pi
        hh = L / n
        z, y, x = np.meshgrid(*(np.arange(n) * hh,) * 3, indexing="ij")
        f = np.sin(x) * np.cos(2 * y) + np.sin(z)
        gx, gy, gz = fd.gradient(f, (hh,) * 3, N)
        e = max(np.abs(gx - np.cos(x) * np.cos(2 * y)).max(),
                np.abs(gy + 2 * np.sin(x) * np.sin(2 * y)).max(),
                np.abs(gz - np.cos(z)).max())
        errs.append(e)
    order = math.log(errs[0] / errs[1]) / math.log(32 / 24)
    assert order >= 2 * N - 0.3, (errs, order)


def test_vw_gradient_form_of_a_plane_wave():
    """u = a + c cos(k x): grad_h u = -c g(k) sin(k x) with g(k) = sum_p 2 w~_p
    sin(p k h) / h, so (lambda/2) h^3 sum |grad_h u|^2 = (lambda/2) |Omega| c^2
    g^2 / 2; as h -> 0 it tends to the continuum (lambda/2) |Omega| c^2 k^2 / 2."""
    N, lam, a, c = 6, 0.2, 1.3, 0.4
    for n in (16, 24):
        L = 7.5
        hh = L / n
        k = 2 * math.pi * 3 / L
        z, y, x = np.meshgrid(*(np.arange(n) * hh,) * 3, indexing="ij")
        u = a + c * np.cos(k * x)
        w = [float(v) for v in fd.gradient_weights_exact(N)]
        g = sum(2 * w[p - 1] * math.sin(p * k * hh) for p in range(1, N + 1)) / hh
        want = 0.5 * lam * L ** 3 * c * c * g * g / 2
        got = energy.vw_gradient_form(u, (hh,) * 3, lam, N)
        assert abs(got - want) <= 1e-12 * want
        assert abs(got - 0.5 * lam * L ** 3 * c * c * k * k / 2) <= 2e-3 * want


def _cell(n, sigma):
    return inputs.cubic_workload(1, n, 1, jitter=0.05, sigma=sigma)


@pytest.mark.parametrize("sigma", [0.8, 1.2])
def test_appendix_b_grid_form_converges_to_the_gaussian_closed_form(sigma):
    """With Gaussian reference charges the grid E_c equals E_c(s) - E_c(s_ref)
    of the pair sums up to the discretisation error, which must shrink with
    h; the forces likewise."""
    s_ref = 0.55
    errs, ferrs = [], []
    for n in (16, 24, 32):
        w = _cell(n, sigma)
        atoms = np.array(w.cell.atoms)
        cut = 8.5 * max(sigma, s_ref)
        e, f, _ = energy.overlap_appendix_b(w.b, atoms, -3.0, sigma, s_ref, w.cell.h, cut)
        box = [m * hh for m, hh in zip(w.b.shape[::-1], w.cell.h)]
        e1, f1 = energy.overlap(atoms, -3.0, sigma, box)
        e2, f2 = energy.overlap(atoms, -3.0, s_ref, box)
        errs.append(abs(e - (e1 - e2)))
        ferrs.append(np.abs(f - (f1 - f2)).max())
    assert errs[1] < errs[0] / 30 and errs[2] < errs[1] / 10, errs
    assert errs[2] <= 1e-6 and ferrs[1] <= 1e-9 and ferrs[2] <= 1e-11, (errs, ferrs)


def test_appendix_b_forces_are_minus_the_grid_energy_gradient():
    sigma, s_ref, n = 1.2, 0.55, 24
    w = _cell(n, sigma)
    atoms = np.array(w.cell.atoms) + np.array([[0.3, -0.2, 0.1], [0.0, 0.25, -0.15],
                                               [-0.1, 0.0, 0.2], [0.2, 0.1, 0.0]])
    cut = 8.5 * sigma

    def e_of(at):
        c = dataclasses.replace(w.cell, atoms=at)
        b = inputs.pseudocharge(c, sigma)
        return energy.overlap_appendix_b(b, at, -3.0, sigma, s_ref, w.cell.h, cut)

    _, f, _ = e_of(atoms)
    d = 1e-4
    for J in (0, 3):
        for a in range(3):
            ap, am = atoms.copy(), atoms.copy()
            ap[J, a] += d
            am[J, a] -= d
            g = (e_of(ap)[0] - e_of(am)[0]) / (2 * d)
            assert abs(-g - f[J, a]) <= 2e-7 * np.abs(f).max(), (J, a, -g, f[J, a])
