"""The density update U(v) (Section 3.3 fixed-point map; Appendix C, Algorithm 1).

For a fixed potential v, U(v) minimises over u >= 0 with h^3 sum u^2 = N_e
  E(u) = h^3 sum [ C_F rho^{5/3} + eps_xc(rho) rho + v rho ] - (lambda/2) h^3 sum u L_h u,
rho = u^2.  Its gradient in the h^3 inner product is 2 H u with
  H u = -(lambda/2) L_h u + (V_TF + V_xc + v) u,
so the Euler-Lagrange equation is H u = eta u (Section 3.3).

The von Weizsacker term uses u L_h u, so that the gradient of the discrete
energy is exactly 2 H u with the FD Laplacian in H (Section 3.3).

Algorithm 1 (Polak-Ribiere non-linear CG with restarts, Brent line search,
renormalisation to N_e), in the paper's order:
  eta_q = <u_q, H u_q> / N_e
  r_q   = -2 (H u_q - eta_q u_q)
  xi    = <r_q - r_{q-1}, r_q> / <r_{q-1}, r_{q-1}>
  d_q   = r_q if q is a multiple of N_restart or xi <= 0, else r_q + xi d_{q-1}
  s     = argmin_s E( sqrt(N_e) (u_q + s d_q) / ||u_q + s d_q|| )    (Brent)
  u_{q+1} = sqrt(N_e) (u_q + s d_q) / ||u_q + s d_q||
The search runs along d_q (the printed listing shows r_q, which would leave
the Polak-Ribiere direction unused); all norms are h^3-weighted.
Stops when ||H u - eta u|| / ||u|| <= tol.

Hartree inside (the paper's own map U(V_LR), Section 3.3 fixed point in the
kernel potential): with pseudocharges b given, the functional also holds the
electrostatic energy 1/2 h^3 sum (rho + b) phi[rho], phi[rho] the zero-mean
solution of -L_h phi = 4 pi (rho + b) (exact, spectral), and v is only the
external part (mu V_LR).  Its gradient is the same 2 (H u - eta u) with phi
added to the potential, because the electrostatic energy is quadratic and
symmetric in rho + b; every evaluation of H (residual, line-search slope)
re-solves phi for the u it is evaluated at.

Line search: Brent's method is applied to the root of the directional
derivative dE/ds (Brent-Dekker root finding after bracketing), which is where
the minimum along the line sits.  A derivative-free search on E(s) itself
cannot locate s much better than sqrt(machine epsilon) because the energy
is flat there, and the outer iteration then stalls near 1e-8.
  dE/ds = 2 <H u(s), u'(s)>,  u'(s) = (sqrt(N_e)/||w||) (d - w <w,d>/||w||^2),
  w = u + s d.
"""
import numpy as np
from scipy.optimize import brentq

from . import fd, poisson, xc


def _dv(h_xyz):
    return float(h_xyz[0] * h_xyz[1] * h_xyz[2])


def energy(u, v, h_xyz, lam, N=6):
    rho = u * u
    dv = _dv(h_xyz)
    local = xc.e_tf(rho) + xc.eps_xc(rho) * rho + v * rho
    return dv * float(local.sum()) - 0.5 * lam * dv * float((u * fd.laplacian(u, h_xyz, N)).sum())


def hamiltonian(u, v, h_xyz, lam, N=6):
    rho = u * u
    return -0.5 * lam * fd.laplacian(u, h_xyz, N) + (xc.v_tf(rho) + xc.v_xc(rho) + v) * u


def el_residual(u, v, h_xyz, lam, n_electrons, N=6):
    """||H u - eta u|| / ||u||, eta = <u, H u> / N_e."""
    hu = hamiltonian(u, v, h_xyz, lam, N)
    eta = _dv(h_xyz) * float((u * hu).sum()) / n_electrons
    return float(np.linalg.norm(hu - eta * u) / np.linalg.norm(u)), eta


def hartree(u, b, h_xyz, N=6):
    """phi[rho]: zero-mean solution of -L_h phi = 4 pi (u^2 + b)."""
    g, _ = poisson.rhs(u * u, b)
    return poisson.solve_exact(g, h_xyz, N)


def update(u0, v, h_xyz, lam, n_electrons, N=6, tol=1e-10, n_restart=50, maxit=20000, b=None):
    """Algorithm 1; returns (u, iterations, final residual, eta).  With b the
    electrostatic energy is part of the functional (phi re-solved for every u)."""
    dv = _dv(h_xyz)
    sqn = np.sqrt(n_electrons)

    def ham(uu):
        vt = v if b is None else v + hartree(uu, b, h_xyz, N)
        return hamiltonian(uu, vt, h_xyz, lam, N)

    def inner(a, b):
        return dv * float((a * b).sum())

    def normalise(w):
        return sqn * w / np.sqrt(inner(w, w))

    u = normalise(np.asarray(u0, dtype=np.float64))
    r_prev = d_prev = None
    s_prev = None
    res = np.inf
    eta = 0.0
    q = 0
    while q < maxit:
        hu = ham(u)
        eta = inner(u, hu) / n_electrons
        r = -2.0 * (hu - eta * u)
        res = float(np.linalg.norm(hu - eta * u) / np.linalg.norm(u))
        if res <= tol:
            break
        xi = inner(r - r_prev, r) / inner(r_prev, r_prev) if r_prev is not None else 0.0
        if q % n_restart == 0 or xi <= 0.0:
            d = r
        else:
            d = r + xi * d_prev

        def slope(s):
            w = u + s * d
            ww = inner(w, w)
            us = sqn * w / np.sqrt(ww)
            dus = (sqn / np.sqrt(ww)) * (d - w * (inner(w, d) / ww))
            return 2.0 * inner(ham(us), dus)

        if slope(0.0) >= 0.0:          # not a descent direction: restart along r
            d = r
        lo, hi = 0.0, (s_prev if s_prev else 1.0 / np.sqrt(max(inner(d, d) / n_electrons, 1e-300)))
        while slope(hi) < 0.0:
            lo, hi = hi, 2.0 * hi
        s = brentq(slope, lo, hi, xtol=1e-15 * hi, rtol=1e-15, maxiter=200)
        u = normalise(u + s * d)
        r_prev, d_prev, s_prev = r, d, (abs(s) if s != 0 else None)
        q += 1
    return u, q, res, eta


def pointwise_minimiser(v, h_xyz, n_electrons, lo=-50.0, hi=50.0):
    """lambda = 0 reference: the minimiser is pointwise.  Each rho(x) solves
    V_TF(rho) + V_xc(rho) + v(x) = eta (or rho = 0 where that is impossible),
    eta fixed by h^3 sum rho = N_e; both found by bisection (brute force)."""
    dv = _dv(h_xyz)

    def rho_of(eta):
        a = np.full(v.shape, 0.0)
        b = np.full(v.shape, 10.0)
        for _ in range(200):
            mid = 0.5 * (a + b)
            f = xc.v_tf(mid) + xc.v_xc(mid) + v - eta
            # V_TF + V_xc is increasing in rho at these densities
            a = np.where(f < 0, mid, a)
            b = np.where(f < 0, b, mid)
        return 0.5 * (a + b)

    for _ in range(200):
        eta = 0.5 * (lo + hi)
        if dv * rho_of(eta).sum() < n_electrons:
            lo = eta
        else:
            hi = eta
    eta = 0.5 * (lo + hi)
    return np.sqrt(rho_of(eta)), eta
