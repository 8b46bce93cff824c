"""Complex shifted equations of the local kernel reformulation (Section 3.1).

-(2 kF)^-2 Lap V + Q V = P f, multiplied through by (2 kF)^2, becomes
(-L_h + kappa) u = f with kappa = (2 kF)^2 Q.  The matrix is complex symmetric
(L_h is real symmetric), nonsingular when kappa is not in the spectrum of L_h.
"""
import numpy as np

from . import fd
from ._clib import lib, ptr


def solve_exact(f: np.ndarray, kappa: complex, h_xyz, N: int = 6) -> np.ndarray:
    """u_hat(k) = f_hat(k) / (-lambda(k) + kappa)."""
    lam = fd.symbol(f.shape, h_xyz, N)
    return np.fft.ifftn(np.fft.fftn(f) / (-lam + kappa))


def apply(u: np.ndarray, kappa: complex, h_xyz, N: int = 6) -> np.ndarray:
    return -fd.laplacian(u.astype(np.complex128), h_xyz, N) + kappa * u


def solve_cocg(f: np.ndarray, kappa: complex, h_xyz, N: int = 6, x0=None,
               tol: float = 1e-12, maxit: int = 100000):
    """Textbook COCG (C oracle); returns (u, iterations, true relative residual)."""
    nz, ny, nx = f.shape
    ff = np.ascontiguousarray(f, dtype=np.complex128)
    u = np.zeros_like(ff) if x0 is None else np.array(x0, dtype=np.complex128, order="C")
    rel = np.zeros(1)
    it = lib().orc_cocg(nx, ny, nz, *map(float, h_xyz), N, float(kappa.real),
                        float(kappa.imag), ptr(ff), ptr(u), float(tol), int(maxit), ptr(rel))
    return u, it, float(rel[0])


def residual(u: np.ndarray, f: np.ndarray, kappa: complex, h_xyz, N: int = 6) -> float:
    r = f - apply(u, kappa, h_xyz, N)
    return float(np.linalg.norm(r) / np.linalg.norm(f))
