"""Ground-state energy terms and forces on the nuclei (test infrastructure:
only tests and the benchmark's CPU leg may use it).

Energy (Section 3.3, the ground-state energy expression; Section 3.2 for the
electrostatic reformulation):
  E = C_F int rho^(5/3) + (lambda/2) int |grad u|^2 + mu T_LR
      + int eps_xc(rho) rho + 1/2 int (rho + b) phi
      - 1/2 sum_J int b_J V_J + E_c,
with rho = u^2, phi the zero-mean solution of -L_h phi = 4 pi (rho + b).
Readings: the von Weizsacker term is the discrete -(lambda/2) h^3 <u, L_h u>
(the form whose gradient is the H u of the density update); T_LR is the
kernel energy of the expansion in use (see oracle.wgc).

Pseudocharges: the stand-in Gaussians b_J = q (2 pi s^2)^(-3/2)
exp(-|x - R_J|^2 / (2 s^2)) summed over periodic images, whose potential is
V_J = q erf(r / (sqrt(2) s)) / r (then -Lap V_J / (4 pi) = b_J).  The self
term and the forces are sums over each atom's grid points within `cut` of
R_J (unwrapped coordinates, so every image is counted once).
Overlap correction (Appendix B): with reference charges that do not overlap,
E_c is the point-charge repulsion minus the Gaussians' own mutual repulsion,
which for Gaussians is the absolutely convergent pair sum
  E_c = 1/2 sum_{I != J, images} q^2 erfc(d_IJ / (2 s)) / d_IJ,
and f^c_J = -dE_c/dR_J.
Forces (Section 3.3):
  f_J = sum_images int grad b_J (phi - V_J) + f^c_J.

Paper forms (Section 3.3 energy expression as printed; Section 4 FD
gradient; Appendix B):
  * vw_gradient_form: (lambda/2) h^3 sum |grad_h u|^2 with the FD gradient;
  * overlap_appendix_b: reference charges b~_J (Gaussians of width s_ref,
    charge q), V_c the zero-mean solution of -L_h V_c = 4 pi (b~ - b) plus
    the constant that makes its mean the mean of sum_J (V~_J - V_J), which
    for Gaussians is -2 pi q M (s_ref^2 - s^2) / |Omega| (the k = 0 limit of
    the pair's potential: its integral is -(2 pi / 3) times the second
    moment of b~_J - b_J);
      E_c = 1/2 h^3 sum (b~ + b) V_c + 1/2 sum_J h^3 sum b_J V_J
            - 1/2 sum_J h^3 sum b~_J V~_J,
      f^c_J = 1/2 sum_images h^3 sum [grad b~_J (V_c - V~_J)
              + grad b_J (V_c + V_J) + (grad V~_J - grad V_J)(b~ + b)
              + b_J grad V_J - b~_J grad V~_J],
    every per-atom sum over the atom's grid points within `cut` (which must
    cover both Gaussians).
"""
import math

import numpy as np
from scipy.special import erf, erfc

from . import fd, poisson, xc


def _atom_points(R, shape, h, cut):
    """Unwrapped grid offsets within `cut` of R: (wrapped flat indices, displacement x - R)."""
    nz, ny, nx = shape
    axes = []
    for a, n in zip(range(3), (nx, ny, nz)):
        i0 = int(math.floor((R[a] - cut) / h[a]))
        i1 = int(math.ceil((R[a] + cut) / h[a]))
        i = np.arange(i0, i1 + 1)
        axes.append((np.mod(i, n), i * h[a] - R[a]))
    (ix, dx), (iy, dy), (iz, dz) = axes
    DZ, DY, DX = np.meshgrid(dz, dy, dx, indexing="ij")
    IZ, IY, IX = np.meshgrid(iz, iy, ix, indexing="ij")
    r = np.sqrt(DX ** 2 + DY ** 2 + DZ ** 2)
    m = r <= cut
    flat = (IZ[m] * ny + IY[m]) * nx + IX[m]
    return flat, np.stack([DX[m], DY[m], DZ[m]], -1), r[m]


def gauss_b(r, q, s):
    return q * (2.0 * math.pi * s * s) ** -1.5 * np.exp(-r * r / (2.0 * s * s))


def gauss_v(r, q, s):
    small = r < 1e-12
    rr = np.where(small, 1.0, r)
    return np.where(small, q * math.sqrt(2.0 / math.pi) / s, q * erf(rr / (math.sqrt(2.0) * s)) / rr)


def self_and_forces(phi, atoms, q, s, h, cut):
    """(-1/2 sum_J h^3 sum b_J V_J, [f_J without the overlap correction])."""
    dv = float(np.prod(h))
    flat_phi = phi.reshape(-1)
    e_self = 0.0
    forces = np.zeros((len(atoms), 3))
    for J, R in enumerate(atoms):
        idx, d, r = _atom_points(R, phi.shape, h, cut)
        b = gauss_b(r, q, s)
        v = gauss_v(r, q, s)
        e_self -= 0.5 * dv * float(np.sum(b * v))
        grad_b = -b[:, None] * d / (s * s)
        forces[J] = dv * np.sum(grad_b * (flat_phi[idx] - v)[:, None], axis=0)
    return e_self, forces


def overlap(atoms, q, s, box, rc=None):
    """(E_c, f^c): erfc pair sums over all images within rc (default 12 s)."""
    rc = 12.0 * s if rc is None else rc
    atoms = np.asarray(atoms, dtype=float)
    box = np.asarray(box, dtype=float)
    nimg = [int(math.ceil(rc / L)) for L in box]
    e = 0.0
    f = np.zeros_like(atoms)
    shifts = [np.array([i, j, k]) * box for i in range(-nimg[0], nimg[0] + 1)
              for j in range(-nimg[1], nimg[1] + 1) for k in range(-nimg[2], nimg[2] + 1)]
    for I in range(len(atoms)):
        for J in range(len(atoms)):
            for t in shifts:
                dvec = atoms[J] + t - atoms[I]
                d = float(np.sqrt(dvec @ dvec))
                if d == 0.0 or d > rc:
                    continue
                e += 0.5 * q * q * erfc(d / (2.0 * s)) / d
                # -d/dR_I of q^2 erfc(d/2s)/d (the pair appears twice in the sum)
                g = q * q * (erfc(d / (2.0 * s)) / d ** 2 + math.exp(-d * d / (4 * s * s)) / (s * math.sqrt(math.pi) * d))
                f[I] -= g * dvec / d
    return e, f


def energy_terms(u, b, h, lam, atoms, q, s, cut, t_lr=0.0, mu=0, N=6):
    """Dict of the energy terms and their total; phi solved here (exact)."""
    dv = float(np.prod(h))
    rho = u * u
    g, _ = poisson.rhs(rho, b)
    phi = poisson.solve_exact(g, h, N)
    out = {
        "tf": dv * float(np.sum(xc.e_tf(rho))),
        "vw": -0.5 * lam * dv * float(np.sum(u * fd.laplacian(u, h, N))),
        "xc": dv * float(np.sum(xc.eps_xc(rho) * rho)),
        "electrostatic": 0.5 * dv * float(np.sum((rho + b) * phi)),
        "kernel": mu * t_lr,
    }
    out["self"], _ = self_and_forces(phi, atoms, q, s, h, cut)
    box = [n * hh for n, hh in zip(u.shape[::-1], h)]
    out["overlap"], _ = overlap(atoms, q, s, box)
    out["total"] = sum(out.values())
    return out, phi


def forces(phi, atoms, q, s, h, cut):
    box = [n * hh for n, hh in zip(phi.shape[::-1], h)]
    _, f = self_and_forces(phi, atoms, q, s, h, cut)
    return f + overlap(atoms, q, s, box)[1]


def gauss_dv(r, q, s):
    """dV/dr of V = q erf(r / (sqrt 2 s)) / r (0 at r = 0)."""
    small = r < 1e-12
    rr = np.where(small, 1.0, r)
    d = q * (math.sqrt(2.0 / math.pi) * np.exp(-rr * rr / (2.0 * s * s)) / (s * rr)
             - erf(rr / (math.sqrt(2.0) * s)) / (rr * rr))
    return np.where(small, 0.0, d)


def vw_gradient_form(u, h, lam, N=6):
    """(lambda/2) h^3 sum |grad_h u|^2 (Section 4 FD gradient)."""
    dv = float(np.prod(h))
    gx, gy, gz = fd.gradient(u, h, N)
    return 0.5 * lam * dv * float(np.sum(gx * gx + gy * gy + gz * gz))


def reference_charge(atoms, shape, h, q, s_ref, cut):
    """b~ on the grid: the Gaussians of width s_ref over each atom's points within cut."""
    bt = np.zeros(int(np.prod(shape)))
    for R in atoms:
        idx, _, r = _atom_points(R, shape, h, cut)
        np.add.at(bt, idx, gauss_b(r, q, s_ref))
    return bt.reshape(shape)


def overlap_appendix_b(b, atoms, q, s, s_ref, h, cut, N=6):
    """(E_c, f^c [M x 3], V_c) by the grid form of Appendix B."""
    shape = b.shape
    dv = float(np.prod(h))
    volume = dv * b.size
    atoms = np.asarray(atoms, dtype=float)
    bt = reference_charge(atoms, shape, h, q, s_ref, cut)
    g, _ = poisson.rhs(bt, -b)
    vc = poisson.solve_exact(g, h, N) - 2.0 * math.pi * q * len(atoms) * (s_ref ** 2 - s ** 2) / volume
    e = 0.5 * dv * float(np.sum((bt + b) * vc))
    f = np.zeros_like(atoms)
    vcf, btf, bf = vc.reshape(-1), bt.reshape(-1), b.reshape(-1)
    for J, R in enumerate(atoms):
        idx, d, r = _atom_points(R, shape, h, cut)
        bj, vj = gauss_b(r, q, s), gauss_v(r, q, s)
        btj, vtj = gauss_b(r, q, s_ref), gauss_v(r, q, s_ref)
        e += 0.5 * dv * float(np.sum(bj * vj)) - 0.5 * dv * float(np.sum(btj * vtj))
        rr = np.where(r < 1e-12, 1.0, r)[:, None]
        unit = d / rr
        grad_b = -bj[:, None] * d / (s * s)
        grad_bt = -btj[:, None] * d / (s_ref * s_ref)
        grad_v = gauss_dv(r, q, s)[:, None] * unit
        grad_vt = gauss_dv(r, q, s_ref)[:, None] * unit
        tot = (btf[idx] + bf[idx])[:, None]
        integrand = (grad_bt * (vcf[idx] - vtj)[:, None] + grad_b * (vcf[idx] + vj)[:, None]
                     + (grad_vt - grad_v) * tot + bj[:, None] * grad_v - btj[:, None] * grad_vt)
        f[J] = 0.5 * dv * np.sum(integrand, axis=0)
    return e, f, vc
