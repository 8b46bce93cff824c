"""Kernel-potential terms of the linear-response functional, K_00 only (L = 0).

Section 3.1 with m = n = p = q = 0 (C_0000 = 1) and R = 4 rational terms:
  V_LR = C_F sum_r [ alpha rho^(alpha-1) V_{beta,r} + beta rho^(beta-1) V_{alpha,r} ]
where V_{beta,r} solves  -(2kF)^-2 Lap V + Q_r V = P_r f_beta,
f_beta = -(2kF)^-2 Lap rho^beta (the m = n = 0 case), and likewise for alpha.
Multiplying by (2kF)^2: (-L_h + kappa_r) V = P_r (-L_h rho^beta), kappa_r = (2kF)^2 Q_r.
The definitions of V_{..beta} (convolution of K with u^{2(n-q+beta)}) fix which
power feeds which equation; the paper's equation labels are read as swapped.
Table of Appendix A: r = 1, 3 given; r = 2, 4 are complex conjugates.
kF = (3 pi^2 rho_bar)^(1/3), rho_bar = N_e / |Omega|.  alpha, beta from Section 5.

System order used everywhere: j = 0..3 -> (beta, r = 1..4); j = 4..7 -> (alpha, r = 1..4).
"""
import math

import numpy as np

from . import fd, helmholtz
from .xc import C_F

ALPHA = 5.0 / 6.0 + math.sqrt(5.0) / 6.0
BETA = 5.0 / 6.0 - math.sqrt(5.0) / 6.0
P00 = (0.108403 + 0.079657j, 0.108403 - 0.079657j, -0.908403 + 0.439708j, -0.908403 - 0.439708j)
Q00 = (-0.470923 - 0.465392j, -0.470923 + 0.465392j, 0.066051 - 0.259678j, 0.066051 + 0.259678j)


def fermi_wavevector(n_electrons: float, volume: float) -> float:
    return (3.0 * math.pi ** 2 * n_electrons / volume) ** (1.0 / 3.0)


def shifts(n_electrons: float, volume: float):
    """kappa_j for the 8 systems (order: beta r=1..4, alpha r=1..4)."""
    k2 = (2.0 * fermi_wavevector(n_electrons, volume)) ** 2
    ks = [k2 * q for q in Q00]
    return np.array(ks + ks)


def rhs(rho: np.ndarray, h_xyz, N: int = 6):
    """The 8 right-hand sides P_r (-L_h rho^p), p = beta for j < 4, alpha after."""
    lb = -fd.laplacian(rho ** BETA, h_xyz, N)
    la = -fd.laplacian(rho ** ALPHA, h_xyz, N)
    return [P00[r] * lb for r in range(4)] + [P00[r] * la for r in range(4)]


def potential(rho: np.ndarray, V, rho_floor: float) -> np.ndarray:
    """V_LR from the 8 solutions (real part; conjugate pairs make it real)."""
    rc = np.maximum(rho, rho_floor)
    vb = sum(V[j] for j in range(4))
    va = sum(V[j] for j in range(4, 8))
    return np.real(C_F * (ALPHA * rc ** (ALPHA - 1.0) * vb + BETA * rc ** (BETA - 1.0) * va))


def solve_all(rho: np.ndarray, h_xyz, n_electrons: float, volume: float, N: int = 6):
    """Exact (spectral) solutions of the 8 shifted systems."""
    ks = shifts(n_electrons, volume)
    fs = rhs(rho, h_xyz, N)
    return [helmholtz.solve_exact(fs[j], ks[j], h_xyz, N) for j in range(8)]
