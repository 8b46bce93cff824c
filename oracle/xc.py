"""Pointwise energy densities and potentials (Sections 2 and 3.3).

Thomas-Fermi: energy C_F rho^{5/3}, potential V_TF = (5/3) C_F rho^{2/3},
C_F = (3/10)(3 pi^2)^{2/3}.
Exchange (LDA): eps_x = -(3/4)(3/pi)^{1/3} rho^{1/3}, V_x = -(3/pi)^{1/3} rho^{1/3}.
Correlation (Perdew-Zunger fit of Ceperley-Alder), r_s = (3/(4 pi rho))^{1/3}:
  r_s >= 1: eps_c = g1 / (1 + b1 sqrt(r_s) + b2 r_s),
            V_c = (g1 + 7/6 g1 b1 sqrt(r_s) + 4/3 g1 b2 r_s) / (1 + b1 sqrt(r_s) + b2 r_s)^2
  r_s <  1: eps_c = A1 ln r_s + B1 + C1 r_s ln r_s + D1 r_s,
            V_c = (A1 + 2/3 C1 r_s) ln r_s + (B1 - A1/3) + 1/3 (2 D1 - C1) r_s
All functions take rho = u^2 >= 0 (arrays).
"""
import numpy as np

C_F = 0.3 * (3.0 * np.pi ** 2) ** (2.0 / 3.0)
GAMMA1, BETA1, BETA2 = -0.1423, 1.0529, 0.3334
A1, B1, C1, D1 = 0.0311, -0.048, 0.002, -0.0116


def e_tf(rho):
    return C_F * rho ** (5.0 / 3.0)


def v_tf(rho):
    return (5.0 / 3.0) * C_F * rho ** (2.0 / 3.0)


def rs(rho):
    return (3.0 / (4.0 * np.pi * rho)) ** (1.0 / 3.0)


def eps_x(rho):
    return -0.75 * (3.0 / np.pi) ** (1.0 / 3.0) * rho ** (1.0 / 3.0)


def v_x(rho):
    return -(3.0 / np.pi) ** (1.0 / 3.0) * rho ** (1.0 / 3.0)


def eps_c(rho):
    r = rs(rho)
    hi = GAMMA1 / (1.0 + BETA1 * np.sqrt(r) + BETA2 * r)
    lo = A1 * np.log(r) + B1 + C1 * r * np.log(r) + D1 * r
    return np.where(r >= 1.0, hi, lo)


def v_c(rho):
    r = rs(rho)
    sq = np.sqrt(r)
    hi = (GAMMA1 + 7.0 / 6.0 * GAMMA1 * BETA1 * sq + 4.0 / 3.0 * GAMMA1 * BETA2 * r) / \
        (1.0 + BETA1 * sq + BETA2 * r) ** 2
    lo = (A1 + 2.0 / 3.0 * C1 * r) * np.log(r) + (B1 - A1 / 3.0) + (2.0 * D1 - C1) * r / 3.0
    return np.where(r >= 1.0, hi, lo)


def eps_xc(rho):
    return eps_x(rho) + eps_c(rho)


def v_xc(rho):
    return v_x(rho) + v_c(rho)
