"""One step of the fixed-point iteration (Section 3.3, flowchart; Appendix D).

The mixing variable is v = phi + mu V_LR, so that the inner map U(v) is a local
minimisation (Algorithm 1) with no solve inside, and each step costs one
Poisson solve plus (for mu = 1) the 8 shifted kernel solves:
  u_k      = U(v_k)
  phi      = Poisson(4 pi (u_k^2 + b))
  V_LR     = kernel potential from the 8 shifted solves (mu = 1 only)
  vhat_k   = phi + mu V_LR
  f_k      = vhat_k - v_k,  reported error ||f_k|| / ||v_k||
  v_{k+1}  = Anderson(v_k, f_k)
Start: u_0 = sqrt(rho_0), v_0 = phi[u_0] + mu V_LR[u_0].
Solves here are the exact discrete solutions (spectral).
"""
import dataclasses

import numpy as np

from . import density, kernel, poisson
from .anderson import Anderson


@dataclasses.dataclass
class Params:
    lam: float = 0.2          # von Weizsacker weight (TFW: 1/5)
    mu: int = 0               # 1 adds the K_00 kernel term
    history: int = 7
    zeta: float = 0.3
    N: int = 6
    u_tol: float = 1e-10
    n_restart: int = 50


def potential_map(u, b, h_xyz, n_electrons, volume, p: Params):
    rho = u * u
    g, _ = poisson.rhs(rho, b)
    phi = poisson.solve_exact(g, h_xyz, p.N)
    v = phi.copy()
    if p.mu:
        V = kernel.solve_all(rho, h_xyz, n_electrons, volume, p.N)
        rho_bar = n_electrons / volume
        v = v + p.mu * kernel.potential(rho, V, 1e-12 * rho_bar)
    return v


class SCF:
    def __init__(self, rho0, b, h_xyz, n_electrons, volume, p: Params):
        self.b, self.h, self.ne, self.vol, self.p = b, h_xyz, n_electrons, volume, p
        self.u = np.sqrt(rho0)
        self.v = potential_map(self.u, b, h_xyz, n_electrons, volume, p)
        self.mixer = Anderson(p.history, p.zeta)

    def step(self):
        p = self.p
        self.u, it, res, eta = density.update(self.u, self.v, self.h, p.lam, self.ne, p.N,
                                              tol=p.u_tol, n_restart=p.n_restart)
        vhat = potential_map(self.u, self.b, self.h, self.ne, self.vol, p)
        f = vhat - self.v
        nv = float(np.linalg.norm(self.v))
        err = float(np.linalg.norm(f)) / nv if nv > 0 else float(np.linalg.norm(f))
        self.v = self.mixer.step(self.v, f).reshape(self.v.shape)
        return err
