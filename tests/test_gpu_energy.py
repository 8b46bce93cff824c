"""Energy terms and forces on the nuclei (Section 3.3; Appendix B overlap
correction) from the SCF context against the oracle, for the Gaussian
stand-in pseudocharges: small cell with displaced atoms (brute-force
overlap images), the 500-atom supercell (binned overlap), TFW and the
kernel functional (K_00 and the order-2 terms)."""
import dataclasses

import numpy as np
import pytest

import paper_1412_8250_amd as ofd
from oracle import energy, wgc
from paper_1412_8250_amd import inputs
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu
SIGMA, CUT = 0.8, 8.5 * 0.8


def _case(which):
    if which == "small":
        w = inputs.small_cell()
        atoms = np.array(w.cell.atoms, dtype=float) + np.array([[0.3, -0.2, 0.1], [0.0, 0.25, -0.15],
                                                                [-0.1, 0.0, 0.2], [0.2, 0.1, 0.0]])
        cell = dataclasses.replace(w.cell, atoms=atoms)
        b = inputs.pseudocharge(cell, SIGMA)
        rho = w.rho * (-b.sum() / w.rho.sum())
        return cell, b, rho, atoms
    w = inputs.supercell_500()
    return w.cell, w.b, w.rho, np.array(w.cell.atoms, dtype=float)


@pytest.mark.parametrize("which,mu,lr", [("small", 0, 0), ("small", 1, 0), ("small", 1, 2), ("supercell", 0, 0)])
def test_energy_and_forces_match_oracle(which, mu, lr):
    torch = torch_cuda()
    announce("energy/forces", which, mu, lr)
    cell, b, rho, atoms = _case(which)
    h, ne, vol = cell.h, cell.n_electrons, cell.volume
    tol = 1e-10
    ctx = ofd.SCF(rho.shape, h, to_dev(b), to_dev(np.sqrt(rho)), ne, lam=0.2 if mu == 0 else 1.0, mu=mu,
                  lr_order=lr, poisson_tol=tol, helmholtz_tol=tol, poisson_mode=ofd.MULTIGRID,
                  helmholtz_precond=ofd.PRECOND_MULTIGRID)
    e_gpu = ctx.energy(atoms, -3.0, SIGMA, CUT)
    f_gpu = ctx.forces(atoms, -3.0, SIGMA, CUT)
    ud = torch.empty(rho.shape, dtype=torch.float64, device="cuda")
    ctx.get(ofd.SCF.U, ud)
    u = to_host(ud)
    t_lr = wgc.energy(u * u, h, ne, vol, L=lr) if mu else 0.0
    e_orc, phi = energy.energy_terms(u, b, h, 0.2 if mu == 0 else 1.0, atoms, -3.0, SIGMA, CUT, t_lr=t_lr, mu=mu)
    f_orc = energy.forces(phi, atoms, -3.0, SIGMA, h, CUT)
    announce("total", e_gpu["total"], e_orc["total"], "max |f|", np.abs(f_orc).max())
    for k in ("tf", "vw", "xc", "electrostatic", "self", "overlap", "kernel", "total"):
        scale = max(1.0, abs(e_orc[k]))
        assert abs(e_gpu[k] - e_orc[k]) <= 1e-8 * scale, (k, e_gpu[k], e_orc[k])
    assert np.abs(f_gpu - f_orc).max() <= 1e-6 * np.abs(f_orc).max() + 1e-9
    ctx.close()


@pytest.mark.parametrize("shape,h,N", [((16, 16, 16), (0.46875,) * 3, 6), ((13, 22, 70), (0.4, 0.45, 0.5), 6),
                                       ((5, 9, 11), (0.3, 0.35, 0.4), 6), ((24, 24, 24), (0.5,) * 3, 3)])
def test_fd_gradient_matches_oracle(shape, h, N):
    """Element by element, including grids shorter than the stencil (repeated wraps)."""
    torch = torch_cuda()
    from oracle import fd
    announce("fd gradient", shape, N)
    x = np.random.default_rng(7).normal(size=shape)
    xd = to_dev(x)
    g = [torch.full_like(xd, float("nan")) for _ in range(3)]
    ofd.fd_gradient_apply(xd, *g, h, N)
    torch.cuda.synchronize()
    ref = fd.gradient(x, h, N)
    for a in range(3):
        scale = np.abs(ref[a]).max()
        assert np.abs(to_host(g[a]) - ref[a]).max() <= 1e-13 * scale, a


def test_fd_gradient_rejects_aliased_outputs():
    torch = torch_cuda()
    x = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(ofd.OfdftError):
        ofd.fd_gradient_apply(x, y, y, torch.zeros_like(x), (0.5,) * 3)


@pytest.mark.parametrize("which,sigma", [("small", 0.8), ("small", 1.2), ("supercell", 1.2)])
def test_paper_form_energy_and_forces_match_oracle(which, sigma):
    """The gradient-form von Weizsacker term and the Appendix B grid-form
    overlap correction (its Poisson solve by the context's multigrid CG to
    1e-12) against the oracle's: the small cell with displaced atoms (the
    reference charge summed over every image) and the 500-atom supercell
    (the cell-list gather)."""
    torch = torch_cuda()
    announce("paper-form energy", which, sigma)
    s_ref, N = 0.55, 6
    cut = 8.5 * max(sigma, s_ref)
    if which == "small":
        w = inputs.cubic_workload(1, 24, 1, jitter=0.05, sigma=sigma)
        atoms = np.array(w.cell.atoms, dtype=float) + np.array([[0.3, -0.2, 0.1], [0.0, 0.25, -0.15],
                                                                [-0.1, 0.0, 0.2], [0.2, 0.1, 0.0]])
    else:
        w = inputs.cubic_workload(5, 96, 2, jitter=0.05, sigma=sigma)
        atoms = np.array(w.cell.atoms, dtype=float)
    cell = dataclasses.replace(w.cell, atoms=atoms)
    b = inputs.pseudocharge(cell, sigma)
    rho = w.rho * (-b.sum() / w.rho.sum())
    h = cell.h
    ctx = ofd.SCF(rho.shape, h, to_dev(b), to_dev(np.sqrt(rho)), cell.n_electrons, lam=0.2, poisson_tol=1e-12,
                  poisson_mode=ofd.MULTIGRID)
    e_gpu = ctx.energy_paper_form(atoms, s_ref, -3.0, sigma, cut)
    f_gpu = ctx.forces_paper_form(atoms, s_ref, -3.0, sigma, cut)
    e_std = ctx.energy(atoms, -3.0, sigma, cut)
    ud = torch.empty(rho.shape, dtype=torch.float64, device="cuda")
    ctx.get(ofd.SCF.U, ud)
    u = to_host(ud)
    vw = energy.vw_gradient_form(u, h, 0.2, N)
    ec, fc, _ = energy.overlap_appendix_b(b, atoms, -3.0, sigma, s_ref, h, cut, N)
    e_orc, phi = energy.energy_terms(u, b, h, 0.2, atoms, -3.0, sigma, cut)
    f_orc = energy.self_and_forces(phi, atoms, -3.0, sigma, h, cut)[1] + fc
    announce("vw", e_gpu["vw"], vw, "E_c", e_gpu["overlap"], ec, "closed", e_std["overlap"])
    assert abs(e_gpu["vw"] - vw) <= 1e-11 * abs(vw)
    assert abs(e_gpu["overlap"] - ec) <= 1e-9 * max(abs(ec), 1e-3)
    # the untouched terms are those of the standard form
    for k in ("tf", "xc", "electrostatic", "self", "kernel"):
        assert e_gpu[k] == e_std[k], k
    assert abs(e_gpu["total"] - (e_std["total"] - e_std["vw"] - e_std["overlap"] + vw + ec)) <= 1e-9 * abs(e_std["total"])
    assert np.abs(f_gpu - f_orc).max() <= 1e-7 * np.abs(f_orc).max() + 1e-10
    ctx.close()
