"""Kernel energy and potential of the linear-response functional expanded to
order L = 2 about the mean density (test infrastructure: only tests and the
benchmark's CPU leg may use it).

Section 2 (linearised kernel energy):
  T_LR = C_F sum_{m,n} sum_{p<=m} sum_{q<=n} C_mnpq
             <rho^(m-p+alpha), K_mn rho^(n-q+beta)>,
  C_mnpq = (-1)^(p+q) / (m! n!) binom(m,p) binom(n,q) rho_bar^(p+q-m-n).
Section 3.1 (local reformulation): K_mn applied to g is sum_r V_r with
  -(2kF)^-2 Lap V_r + Q_mnr V_r = P_mnr f,
f = -(2kF)^-2 Lap g for m = n = 0 and f = g otherwise; multiplied by
(2kF)^2: (-L_h + kappa_r) V_r = P_r (-L_h g) for K_00 and
(2kF)^2 P_r g for the others, kappa_r = (2kF)^2 Q_mnr.  The potential is the
derivative of T_LR with respect to rho:
  V_LR = C_F sum C_mnpq [ (m-p+alpha) rho^(m-p+alpha-1) K_mn rho^(n-q+beta)
                        + (n-q+beta) rho^(n-q+beta-1) K_mn rho^(m-p+alpha) ].
Appendix A gives P and Q for K_00, K_10, K_20, K_11 (r = 1, 3; r = 2, 4 are
their conjugates; P_mn = P_nm, Q_mn = Q_nm).  Readings: the expansion keeps
the pairs with m + n <= L, the ones the table covers; the Q_11, r = 1 entry
printed with an imaginary part of -0.0266195 (one digit more than every
other entry) is read as -0.266195, in line with the neighbouring second-order
kernel K_20 (-0.233840); the smaller value would put the shift almost on the
real axis inside the spectrum of -L_h, a near-resonant kernel.  That entry
is therefore parity unpinned: no printed number fixes it, and every result
containing K_11 follows the reading.
Convolutions with the same kernel and the same power of rho are computed once.
"""
import math

import numpy as np

from . import fd, helmholtz
from .kernel import ALPHA, BETA, fermi_wavevector
from .xc import C_F

# (P, Q) for r = 1, 3 of each kernel (m, n) with m >= n
TABLE = {
    (0, 0): ((0.108403 + 0.079657j, -0.908403 + 0.439708j), (-0.470923 - 0.465392j, 0.066051 - 0.259678j)),
    (1, 0): ((-0.030515 + 0.015027j, 0.028915 - 0.008817j), (-0.597793 - 0.294130j, -0.087917 - 0.164937j)),
    (2, 0): ((0.008907 - 0.032841j, -0.034974 + 0.009116j), (-0.537986 - 0.233840j, -0.041565 - 0.196662j)),
    (1, 1): ((0.012423 - 0.034421j, -0.031907 + 0.007392j), (-0.511699 - 0.266195j, -0.034031 - 0.188927j)),
}


def kernel_key(m: int, n: int):
    return (max(m, n), min(m, n))


def coefficients(m: int, n: int):
    """P_r, Q_r for r = 1..4 of K_mn."""
    (p1, p3), (q1, q3) = TABLE[kernel_key(m, n)]
    return (p1, np.conj(p1), p3, np.conj(p3)), (q1, np.conj(q1), q3, np.conj(q3))


def pairs(L: int = 2):
    return [(m, n) for m in range(L + 1) for n in range(L + 1) if m + n <= L]


def c_mnpq(m, n, p, q, rho_bar):
    return ((-1.0) ** (p + q) / (math.factorial(m) * math.factorial(n)) * math.comb(m, p) * math.comb(n, q)
            * rho_bar ** (p + q - m - n))


def apply_kernel(m, n, g, h_xyz, n_electrons, volume, N: int = 6):
    """K_mn g by the exact (spectral) solves of the R = 4 shifted equations."""
    k2 = (2.0 * fermi_wavevector(n_electrons, volume)) ** 2
    P, Q = coefficients(m, n)
    f = -fd.laplacian(g, h_xyz, N) if (m, n) == (0, 0) else k2 * g
    out = sum(helmholtz.solve_exact(P[r] * f, k2 * Q[r], h_xyz, N) for r in range(4))
    return np.real(out)


class Convolutions:
    """K_mn rho^a for every (kernel, power) the expansion needs, each once."""

    def __init__(self, rho, h_xyz, n_electrons, volume, L=2, N=6):
        self.rho, self.h, self.ne, self.vol, self.N = rho, h_xyz, n_electrons, volume, N
        self.cache = {}

    def __call__(self, m, n, a):
        key = (kernel_key(m, n), round(a, 12))
        if key not in self.cache:
            self.cache[key] = apply_kernel(m, n, self.rho ** a, self.h, self.ne, self.vol, self.N)
        return self.cache[key]


def energy(rho, h_xyz, n_electrons, volume, L=2, N=6):
    dv = float(np.prod(h_xyz))
    rho_bar = n_electrons / volume
    K = Convolutions(rho, h_xyz, n_electrons, volume, L, N)
    t = 0.0
    for m, n in pairs(L):
        for p in range(m + 1):
            for q in range(n + 1):
                a, b = m - p + ALPHA, n - q + BETA
                t += c_mnpq(m, n, p, q, rho_bar) * dv * float(np.sum(rho ** a * K(m, n, b)))
    return C_F * t


def potential(rho, h_xyz, n_electrons, volume, L=2, N=6, rho_floor=None):
    """V_LR; the prefactor powers use max(rho, rho_floor) (default 1e-12 rho_bar)."""
    rho_bar = n_electrons / volume
    rc = np.maximum(rho, 1e-12 * rho_bar if rho_floor is None else rho_floor)
    K = Convolutions(rho, h_xyz, n_electrons, volume, L, N)
    v = np.zeros_like(rho)
    for m, n in pairs(L):
        for p in range(m + 1):
            for q in range(n + 1):
                a, b = m - p + ALPHA, n - q + BETA
                c = c_mnpq(m, n, p, q, rho_bar)
                v += c * (a * rc ** (a - 1.0) * K(m, n, b) + b * rc ** (b - 1.0) * K(m, n, a))
    return C_F * v


def systems(L=2):
    """The distinct shifted systems, in the order the GPU batch uses:
    for each convolution (kernel (m, n) with m >= n, power a), r = 1 then r = 3.
    Returns a list of (m, n, a, r) with r in {0, 2} (index into the r = 1..4 tables)."""
    conv = []
    for m, n in pairs(L):
        for p in range(m + 1):
            for q in range(n + 1):
                for a in (n - q + BETA, m - p + ALPHA):
                    key = (kernel_key(m, n), round(a, 12))
                    if key not in [(kernel_key(*c[:2]), round(c[2], 12)) for c in conv]:
                        conv.append((kernel_key(m, n)[0], kernel_key(m, n)[1], a))
    return [(m, n, a, r) for (m, n, a) in conv for r in (0, 2)]
