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


def kernel_potential(u, h_xyz, n_electrons, volume, N=6):
    """V_LR[u] from the shifted solves (K_00, Appendix A)."""
    rho = u * u
    V = kernel.solve_all(rho, h_xyz, n_electrons, volume, N)
    return kernel.potential(rho, V, 1e-12 * n_electrons / volume)


class KernelPotentialSCF:
    """The paper's own fixed point (Section 3.3, the map V_LR -> V[U(V_LR)] and
    the flowchart): the mixing variable is the kernel potential V_LR alone and
    U minimises the functional with the electrostatics inside (phi re-solved
    for every u, density.update with b), with mu V_LR as the external
    potential.  Start: u_0 = sqrt(rho_0), V_0 = V_LR[u_0].  Error:
    ||Vhat_k - V_k|| / ||V_k||.  For mu = 0 one step gives the TFW ground
    state and the error is 0."""

    def __init__(self, rho0, b, h_xyz, n_electrons, volume, p: Params):
        self.b, self.h, self.ne, self.vol, self.p = b, h_xyz, n_electrons, volume, p
        self.u = np.sqrt(rho0)
        self.V = (kernel_potential(self.u, h_xyz, n_electrons, volume, p.N) if p.mu
                  else np.zeros_like(self.u))
        self.mixer = Anderson(p.history, p.zeta)

    def step(self):
        p = self.p
        self.u, it, res, eta = density.update(self.u, p.mu * self.V, self.h, p.lam, self.ne, p.N,
                                              tol=p.u_tol, n_restart=p.n_restart, b=self.b)
        if not p.mu:
            return 0.0
        vhat = kernel_potential(self.u, self.h, self.ne, self.vol, p.N)
        f = vhat - self.V
        nv = float(np.linalg.norm(self.V))
        err = float(np.linalg.norm(f)) / nv if nv > 0 else float(np.linalg.norm(f))
        self.V = self.mixer.step(self.V, f).reshape(self.V.shape)
        return err
