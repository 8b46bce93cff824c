"""Seeded synthetic inputs shaped like the paper's aluminium FCC cells.

This module is shared by the GPU path's callers (tests, benchmark, SCF driver)
and by the CPU oracle's tests.  It holds no arithmetic of the method itself:
no finite-difference operator, no solver, no functional.  It only places
atoms, evaluates normalised Gaussian nuclear pseudocharges, draws a smooth
random density and draws complex shifts.

Stand-ins (the paper's Goodwin-Needs-Heine pseudopotential and isolated-atom
densities are not available):

* nuclear charge density b: a normalised Gaussian of standard deviation
  ``sigma`` carrying ``-3`` electrons' worth of charge per Al atom, summed over
  all periodic images (the sign follows the requirement that the electron
  density plus b integrate to zero, Section 3.3, Poisson equation);
* electron density rho = rho_bar (1 + 0.05 g) with g a smooth random field made
  of the Fourier modes k in {0..3}^3 minus the zero mode, scaled to max|g| = 1,
  then rescaled so that h^3 sum(rho) = -h^3 sum(b) (net charge zero).

Grid convention: arrays are ``[nz][ny][nx]`` (x fastest); grid point
(i, j, k) sits at (i*hx, j*hy, k*hz), i = 0..nx-1 (Section 4, uniform grid).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

A_AL = 7.5                       # bohr, FCC lattice constant used by the workloads
Z_AL = 3.0                       # valence electrons per Al atom
FCC_BASIS = np.array([[0.0, 0.0, 0.0],
                      [0.0, 0.5, 0.5],
                      [0.5, 0.0, 0.5],
                      [0.5, 0.5, 0.0]])


@dataclasses.dataclass
class Cell:
    """A periodic orthorhombic cell on a uniform grid."""
    n: Tuple[int, int, int]          # (nx, ny, nz)
    L: Tuple[float, float, float]    # (Lx, Ly, Lz) in bohr
    atoms: np.ndarray                # (M, 3) positions in bohr, inside [0, L)

    @property
    def h(self) -> Tuple[float, float, float]:
        return tuple(L / n for L, n in zip(self.L, self.n))

    @property
    def shape(self) -> Tuple[int, int, int]:
        """numpy shape, z slowest."""
        return (self.n[2], self.n[1], self.n[0])

    @property
    def n_electrons(self) -> float:
        return Z_AL * len(self.atoms)

    @property
    def volume(self) -> float:
        return self.L[0] * self.L[1] * self.L[2]


def fcc_atoms(cells: Sequence[int], a: float, jitter: float,
              rng: np.random.Generator, vacancy: bool = False) -> np.ndarray:
    """FCC lattice of ``cells`` conventional cubes, optionally jittered.

    With ``vacancy`` the atom nearest the box centre is removed (the paper
    removes a central atom for its vacancy runs, Section 5.4).
    """
    c1, c2, c3 = cells
    grid = np.stack(np.meshgrid(np.arange(c1), np.arange(c2), np.arange(c3),
                                indexing="ij"), -1).reshape(-1, 3)
    pos = (grid[:, None, :] + FCC_BASIS[None, :, :]).reshape(-1, 3) * a
    if vacancy:
        centre = 0.5 * a * np.array([c1, c2, c3], dtype=float)
        pos = np.delete(pos, int(np.argmin(((pos - centre) ** 2).sum(1))), axis=0)
    if jitter > 0:
        pos = pos + rng.normal(0.0, jitter, size=pos.shape)
    box = a * np.array([c1, c2, c3], dtype=float)
    return np.mod(pos, box)


def _axis_factor(r: float, n: int, L: float, sigma: float, cut: float):
    """Periodic 1D Gaussian factor exp(-(x-r-mL)^2/(2 sigma^2)) summed over images.

    Returns (indices, values) restricted to grid points within ``cut`` of some
    image of ``r``.
    """
    h = L / n
    i0 = int(math.floor((r - cut) / h))
    i1 = int(math.ceil((r + cut) / h))
    idx = np.arange(i0, i1 + 1)
    vals = np.exp(-((idx * h - r) ** 2) / (2.0 * sigma * sigma))
    full = np.bincount(np.mod(idx, n), weights=vals, minlength=n)
    support = np.unique(np.mod(idx, n))
    return support, full[support]


def pseudocharge(cell: Cell, sigma: float = 0.8, charge: float = -Z_AL,
                 cutoff_sigmas: float = 8.5) -> np.ndarray:
    """Sum of normalised periodic Gaussians, ``charge`` electrons per atom.

    The periodic image sum of an isotropic Gaussian in an orthorhombic box
    factorises into per-axis image sums, which is how it is evaluated here.
    """
    nx, ny, nz = cell.n
    Lx, Ly, Lz = cell.L
    b = np.zeros(cell.shape)
    norm = charge * (2.0 * math.pi * sigma * sigma) ** -1.5
    cut = cutoff_sigmas * sigma
    for (x, y, z) in cell.atoms:
        sx, fx = _axis_factor(x, nx, Lx, sigma, cut)
        sy, fy = _axis_factor(y, ny, Ly, sigma, cut)
        sz, fz = _axis_factor(z, nz, Lz, sigma, cut)
        b[np.ix_(sz, sy, sx)] += norm * (fz[:, None, None] * fy[None, :, None] * fx[None, None, :])
    return b


def smooth_field(n: Sequence[int], rng: np.random.Generator, kmax: int = 3) -> np.ndarray:
    """g = sum_k a_k cos(2 pi k.x/L + theta_k), k in {0..kmax}^3 minus 0, max|g| = 1.

    a_k ~ N(0,1), theta_k ~ U(0, 2 pi), drawn in that order, modes in C order
    of (kz, ky, kx).
    """
    nx, ny, nz = n
    m = kmax + 1
    amp = rng.normal(0.0, 1.0, size=(m, m, m))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=(m, m, m))
    coef = amp * np.exp(1j * phase)
    coef[0, 0, 0] = 0.0
    k = np.arange(m)
    ex = np.exp(2j * math.pi * np.outer(k, np.arange(nx)) / nx)   # [kx, i]
    ey = np.exp(2j * math.pi * np.outer(k, np.arange(ny)) / ny)   # [ky, j]
    ez = np.exp(2j * math.pi * np.outer(k, np.arange(nz)) / nz)   # [kz, l]
    t1 = np.einsum("zyx,xi->zyi", coef, ex)
    t2 = np.einsum("zyi,yj->zji", t1, ey)
    g = np.empty((nz, ny, nx))
    for l in range(nz):
        g[l] = np.real(np.tensordot(ez[:, l], t2, axes=(0, 0)))
    return g / np.abs(g).max()


def electron_density(cell: Cell, b: np.ndarray, rng: np.random.Generator,
                     amplitude: float = 0.05) -> np.ndarray:
    """rho_bar (1 + amplitude g), rescaled so sum(rho) = -sum(b)."""
    rho_bar = cell.n_electrons / cell.volume
    rho = rho_bar * (1.0 + amplitude * smooth_field(cell.n, rng))
    return rho * (-b.sum() / rho.sum())


# ----------------------------------------------------------------------------
# Workload recipes.  Each returns plain numpy arrays; seeds are fixed.
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    cell: Cell
    b: np.ndarray
    rho: np.ndarray


def cubic_workload(cells: int, n: int, seed, jitter: float = 0.0, vacancy: bool = False,
                   a: float = A_AL, sigma: float = 0.8) -> Workload:
    """FCC Al-like cube of ``cells``^3 conventional cells on an n^3 grid."""
    rng = np.random.default_rng(seed)
    atoms = fcc_atoms((cells, cells, cells), a, jitter, rng, vacancy)
    cell = Cell((n, n, n), (cells * a,) * 3, atoms)
    b = pseudocharge(cell, sigma)
    rho = electron_density(cell, b, rng)
    return Workload(cell, b, rho)


def small_cell(seed: int = 1) -> Workload:
    """4-atom FCC cube, a = 7.5 bohr, 16^3 grid (h = 0.46875)."""
    return cubic_workload(1, 16, seed)


def supercell_500(vacancy: bool = False) -> Workload:
    """5x5x5 FCC cells (500 atoms, or 499 with a vacancy), 96^3 grid, jitter 0.05."""
    return cubic_workload(5, 96, 3 if vacancy else 2, jitter=0.05, vacancy=vacancy)


def large_cell(sigma: float = 0.8) -> Workload:
    """16x16x16 FCC cells (16384 atoms), 120 bohr box, 320^3 grid, jitter 0.05."""
    return cubic_workload(16, 320, 5, jitter=0.05, sigma=sigma)


def batched_cell_sizes(count: int = 32, seed: int = 4) -> List[Tuple[int, int]]:
    """(lattice multiples m, grid n) for the uneven batch of cells.

    n is drawn uniformly from {24, 32, ..., 96}; m in {2,3,4,5} is the lattice
    multiple whose spacing m a / n lies in [0.39, 0.63] closest to 0.5.
    """
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.arange(24, 97, 8), size=count)
    out = []
    for n in ns:
        best = None
        for m in (2, 3, 4, 5):
            h = m * A_AL / n
            if 0.385 <= h <= 0.63:
                if best is None or abs(h - 0.5) < abs(best[1] - 0.5):
                    best = (m, h)
        out.append((best[0], int(n)))
    return out


def shifted_system_draws(rng: np.random.Generator, count: int = 8):
    """Complex shifts with |kappa| log-uniform in [0.1, 5], |arg| <= 0.45 pi
    (so Re kappa > 0), and unit-modulus right-hand-side factors c_j."""
    mag = np.exp(rng.uniform(math.log(0.1), math.log(5.0), size=count))
    arg = rng.uniform(-0.45 * math.pi, 0.45 * math.pi, size=count)
    kappa = mag * np.exp(1j * arg)
    c = np.exp(1j * rng.uniform(0.0, 2.0 * math.pi, size=count))
    return kappa, c


def batched_workloads(count: int = 32, seed: int = 4, shifts_per_cell: int = 8):
    """The uneven batch: list of (Workload, kappa[8], c[8]).

    The first half of each cell's shifts take the alpha-power right-hand side,
    the second half the beta-power one.
    """
    out = []
    for ci, (m, n) in enumerate(batched_cell_sizes(count, seed)):
        rng = np.random.default_rng([seed, ci])
        atoms = fcc_atoms((m, m, m), A_AL, 0.05, rng)
        cell = Cell((n, n, n), (m * A_AL,) * 3, atoms)
        b = pseudocharge(cell)
        rho = electron_density(cell, b, rng)
        kappa, c = shifted_system_draws(rng, shifts_per_cell)
        out.append((Workload(cell, b, rho), kappa, c))
    return out


TRAIN_SHAPES = ((4, 64), (4, 80), (5, 80), (5, 96), (6, 96), (6, 112))


def training_workload(i: int) -> Workload:
    """Training cell i (seed 1000 + i): 4^3-6^3 cells, n in {64..112}, jitter 0.1."""
    rng = np.random.default_rng(1000 + i)
    m, n = TRAIN_SHAPES[int(rng.integers(len(TRAIN_SHAPES)))]
    atoms = fcc_atoms((m, m, m), A_AL, 0.1, rng)
    cell = Cell((n, n, n), (m * A_AL,) * 3, atoms)
    b = pseudocharge(cell)
    return Workload(cell, b, electron_density(cell, b, rng))


def heldout_workload(which: int) -> Workload:
    """Held-out cells: 0 -> 5^3 cells on 96^3 (seed 9001); 1 -> 10^3 on 192^3 (seed 9002)."""
    m, n, seed = ((5, 96, 9001), (10, 192, 9002))[which]
    return cubic_workload(m, n, seed, jitter=0.1)


def jellium(cells: int, n: int, a: float = A_AL) -> Workload:
    """Uniform density and uniform neutralising background: a trivial fixed point."""
    atoms = fcc_atoms((cells,) * 3, a, 0.0, np.random.default_rng(0))
    cell = Cell((n, n, n), (cells * a,) * 3, atoms)
    rho_bar = cell.n_electrons / cell.volume
    return Workload(cell, np.full(cell.shape, -rho_bar), np.full(cell.shape, rho_bar))


# ----------------------------------------------------------------------------
# The same recipes evaluated with torch on a device, for workloads that need
# thousands of cells (the learned aid's training pairs).  Every random draw is
# the numpy recipe's own (same generator, same order), so a cell equals its
# numpy counterpart up to rounding; only the evaluation of the Gaussians and
# of the smooth field runs on the device.  Still no arithmetic of the method.
# ----------------------------------------------------------------------------

def _axis_factors_torch(r, n: int, L: float, sigma: float, cut: float, torch, device):
    """[M, n] periodic 1D Gaussian factors, the numpy recipe's window: the
    unwrapped points floor((r - cut)/h) .. ceil((r + cut)/h), folded mod n."""
    h = L / n
    r = torch.as_tensor(r, dtype=torch.float64, device=device)
    i0 = torch.floor((r - cut) / h).to(torch.int64)
    i1 = torch.ceil((r + cut) / h).to(torch.int64)
    width = int(math.ceil(2.0 * cut / h)) + 3
    idx = i0[:, None] + torch.arange(width, device=device)[None, :]
    vals = torch.exp(-((idx.to(torch.float64) * h - r[:, None]) ** 2) / (2.0 * sigma * sigma))
    vals = torch.where(idx <= i1[:, None], vals, torch.zeros_like(vals))
    out = torch.zeros((r.shape[0], n), dtype=torch.float64, device=device)
    return out.scatter_add_(1, torch.remainder(idx, n), vals)


def pseudocharge_torch(cell: Cell, device, sigma: float = 0.8, charge: float = -Z_AL,
                       cutoff_sigmas: float = 8.5):
    """pseudocharge() on a device: the per-axis image sums as [M, n] factors,
    b[z, y, x] = norm sum_J Fz[J, z] Fy[J, y] Fx[J, x] as one matrix product."""
    import torch
    nx, ny, nz = cell.n
    Lx, Ly, Lz = cell.L
    cut = cutoff_sigmas * sigma
    at = cell.atoms
    fx = _axis_factors_torch(at[:, 0], nx, Lx, sigma, cut, torch, device)
    fy = _axis_factors_torch(at[:, 1], ny, Ly, sigma, cut, torch, device)
    fz = _axis_factors_torch(at[:, 2], nz, Lz, sigma, cut, torch, device)
    norm = charge * (2.0 * math.pi * sigma * sigma) ** -1.5
    gyx = (fy[:, :, None] * fx[:, None, :]).reshape(len(at), ny * nx)
    return (norm * (fz.t() @ gyx)).reshape(nz, ny, nx)


def smooth_field_torch(n: Sequence[int], rng: np.random.Generator, device, kmax: int = 3):
    """smooth_field() on a device (same draws, same modes)."""
    import torch
    nx, ny, nz = n
    m = kmax + 1
    amp = rng.normal(0.0, 1.0, size=(m, m, m))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=(m, m, m))
    coef = amp * np.exp(1j * phase)
    coef[0, 0, 0] = 0.0
    k = np.arange(m)
    c = torch.from_numpy(coef).to(device)
    ex = torch.from_numpy(np.exp(2j * math.pi * np.outer(k, np.arange(nx)) / nx)).to(device)
    ey = torch.from_numpy(np.exp(2j * math.pi * np.outer(k, np.arange(ny)) / ny)).to(device)
    ez = torch.from_numpy(np.exp(2j * math.pi * np.outer(k, np.arange(nz)) / nz)).to(device)
    t1 = (c.reshape(m * m, m) @ ex).reshape(m, m, nx)                   # [kz, ky, i]
    t2 = torch.einsum("zyi,yj->zji", t1, ey).reshape(m, ny * nx)        # [kz, (j, i)]
    g = (ez.t() @ t2).real.reshape(nz, ny, nx)
    return g / g.abs().max()


def electron_density_torch(cell: Cell, b, rng: np.random.Generator, device, amplitude: float = 0.05):
    rho_bar = cell.n_electrons / cell.volume
    rho = rho_bar * (1.0 + amplitude * smooth_field_torch(cell.n, rng, device))
    return rho * (-b.sum() / rho.sum())


def training_cell_torch(i: int, device):
    """training_workload(i) on a device: (cell, b, rho) with b, rho tensors."""
    rng = np.random.default_rng(1000 + i)
    m, n = TRAIN_SHAPES[int(rng.integers(len(TRAIN_SHAPES)))]
    atoms = fcc_atoms((m, m, m), A_AL, 0.1, rng)
    cell = Cell((n, n, n), (m * A_AL,) * 3, atoms)
    b = pseudocharge_torch(cell, device)
    return cell, b, electron_density_torch(cell, b, rng, device)


def heldout_cell_torch(which: int, device):
    """heldout_workload(which) on a device: (cell, b, rho)."""
    m, n, seed = ((5, 96, 9001), (10, 192, 9002))[which]
    rng = np.random.default_rng(seed)
    atoms = fcc_atoms((m, m, m), A_AL, 0.1, rng)
    cell = Cell((n, n, n), (m * A_AL,) * 3, atoms)
    b = pseudocharge_torch(cell, device)
    return cell, b, electron_density_torch(cell, b, rng, device)
