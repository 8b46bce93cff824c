"""Reference definition of the multigrid preconditioner cycle (test
infrastructure: only tests and the benchmark's CPU leg may use it).

The paper's conclusion (Section 5.5) asks for a real-space preconditioner
for its CG solves; this is the one the library uses, written out plainly so
the device cycle can be compared value by value.  M r is one V(nu, nu) cycle
for the second-order periodic operator A = -Delta_2 + kappa (7-point stencil,
c_a = 1 / h_a^2) started from zero:
  * pre-smoothing: nu damped Jacobi sweeps  u <- u + omega (r - A u) / (6-point
    diagonal sum 2 (c_x + c_y + c_z) + kappa), the first from u = 0;
  * coarse correction: residual, full weighting (restriction R = P^T / 8:
    weights 1, 1/2, 1/4, 1/8 over the 27 fine points around each even point),
    the cycle on the grid of half the points per axis with c_a / 4, trilinear
    prolongation P (even fine points copy, odd ones average their two coarse
    neighbours per axis) added to u;
  * post-smoothing: nu sweeps;
  * coarsest grid (every axis <= coarse_max): the exact solve of A by the DFT,
    eigenvalues sum_a c_a (2 - 2 cos(2 pi k_a / n_a)) + kappa; a zero
    eigenvalue (kappa = 0, k = 0) gives a zero component.
Pinned in the CPU tests against a dense-matrix construction of the same
cycle and against the exact inverse on one-level grids.
"""
import numpy as np


def apply7(u: np.ndarray, c_xyz, kappa: complex = 0.0) -> np.ndarray:
    """A u for the periodic 7-point operator; arrays are (z, y, x)."""
    cx, cy, cz = c_xyz
    out = (2.0 * (cx + cy + cz) + kappa) * u
    for axis, ca in ((2, cx), (1, cy), (0, cz)):
        out = out - ca * (np.roll(u, 1, axis) + np.roll(u, -1, axis))
    return out


def restrict(r: np.ndarray) -> np.ndarray:
    """Full weighting onto the even points (every axis halved)."""
    w = {-1: 0.5, 0: 1.0, 1: 0.5}
    out = np.zeros(tuple(n // 2 for n in r.shape), dtype=r.dtype)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                shifted = np.roll(r, (-dz, -dy, -dx), (0, 1, 2))    # shifted[i] = r[i + d]
                out = out + w[dz] * w[dy] * w[dx] * shifted[::2, ::2, ::2]
    return out / 8.0


def prolong(uc: np.ndarray) -> np.ndarray:
    """Trilinear interpolation onto the grid of twice the points per axis."""
    out = uc
    for axis in range(3):
        n = out.shape[axis] * 2
        shape = list(out.shape)
        shape[axis] = n
        fine = np.zeros(shape, dtype=out.dtype)
        even = [slice(None)] * 3
        odd = [slice(None)] * 3
        even[axis] = slice(0, None, 2)
        odd[axis] = slice(1, None, 2)
        fine[tuple(even)] = out
        fine[tuple(odd)] = 0.5 * (out + np.roll(out, -1, axis))
        out = fine
    return out


def coarse_solve(f: np.ndarray, c_xyz, kappa: complex = 0.0) -> np.ndarray:
    nz, ny, nx = f.shape
    cx, cy, cz = c_xyz
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lam = (cx * (2 - 2 * np.cos(2 * np.pi * kx / nx)) + cy * (2 - 2 * np.cos(2 * np.pi * ky / ny))
           + cz * (2 - 2 * np.cos(2 * np.pi * kz / nz)) + kappa)
    fh = np.fft.fftn(f)
    with np.errstate(divide="ignore", invalid="ignore"):
        uh = np.where(lam == 0, 0.0, fh / np.where(lam == 0, 1.0, lam))
    u = np.fft.ifftn(uh)
    return u.real if np.isrealobj(f) else u


def vcycle(r: np.ndarray, h_xyz, kappa: complex = 0.0, nu: int = 2, omega: float = 0.8,
           coarse_max: int = 16) -> np.ndarray:
    """M r for grid spacing h (x, y, z order); r is (z, y, x)."""
    return _cycle(r, [1.0 / h ** 2 for h in h_xyz], kappa, nu, omega, coarse_max)


def _cycle(f, c, kappa, nu, omega, coarse_max):
    if max(f.shape) <= coarse_max:
        return coarse_solve(f, c, kappa)
    if any(n % 2 for n in f.shape):
        raise ValueError("grid cannot be halved")
    diag = 2.0 * sum(c) + kappa
    u = omega * f / diag
    for _ in range(1, nu):
        u = u + omega * (f - apply7(u, c, kappa)) / diag
    r = f - apply7(u, c, kappa)
    u = u + prolong(_cycle(restrict(r), [ca / 4.0 for ca in c], kappa, nu, omega, coarse_max))
    for _ in range(nu):
        u = u + omega * (f - apply7(u, c, kappa)) / diag
    return u
