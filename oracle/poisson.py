"""Periodic Poisson problem for the electrostatic potential (Section 3.3).

-(1/4 pi) Lap phi = rho + b, periodic; well-posed because the net charge is
zero; the free constant is fixed by a zero integral (Section 4).  Discretely:
the unique phi with -L_h phi = P g, sum(phi) = 0, g = 4 pi (rho + b),
P = I - (1/n) 1 1^T.
"""
import numpy as np

from . import fd
from ._clib import lib, ptr


def rhs(rho: np.ndarray, b: np.ndarray):
    """g = 4 pi (rho + b) projected to zero mean; returns (g, removed_mean)."""
    g = 4.0 * np.pi * (rho + b)
    m = g.mean()
    return g - m, m


def solve_exact(g: np.ndarray, h_xyz, N: int = 6) -> np.ndarray:
    """The discrete solution by diagonalising L_h with the DFT:
    phi_hat(k) = g_hat(k) / (-lambda(k)), phi_hat(0) = 0."""
    lam = fd.symbol(g.shape, h_xyz, N)
    gh = np.fft.fftn(g)
    lam[0, 0, 0] = 1.0
    ph = gh / (-lam)
    ph[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(ph))


def solve_cg(g: np.ndarray, h_xyz, N: int = 6, x0=None, tol: float = 1e-12,
             maxit: int = 100000):
    """Textbook CG (C oracle); returns (phi, iterations, true relative residual)."""
    nz, ny, nx = g.shape
    gg = np.ascontiguousarray(g, dtype=np.float64)
    x = np.zeros_like(gg) if x0 is None else np.array(x0, dtype=np.float64, order="C")
    rel = np.zeros(1)
    it = lib().orc_cg_poisson(nx, ny, nz, *map(float, h_xyz), N, ptr(gg), ptr(x),
                              float(tol), int(maxit), ptr(rel))
    return x, it, float(rel[0])


def residual(phi: np.ndarray, g: np.ndarray, h_xyz, N: int = 6) -> float:
    """||P g + L_h phi|| / ||P g|| with the oracle stencil in FP64."""
    pg = g - g.mean()
    r = pg + fd.laplacian(phi, h_xyz, N)
    return float(np.linalg.norm(r) / np.linalg.norm(pg))
