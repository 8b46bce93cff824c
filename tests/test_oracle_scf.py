"""Pins of the fixed-point step (Section 3.3 fixed-point iteration; Appendix D)."""
import numpy as np

from oracle import density, kernel, poisson, scf
from paper_1412_8250_amd import inputs


def test_jellium_is_a_fixed_point():
    j = inputs.jellium(1, 12)
    for mu, lam in ((0, 0.2), (1, 1.0)):
        s = scf.SCF(j.rho, j.b, j.cell.h, j.cell.n_electrons, j.cell.volume,
                    scf.Params(lam=lam, mu=mu))
        assert np.abs(s.v).max() < 1e-12
        assert s.step() < 1e-12 or np.linalg.norm(s.v) == 0.0


def test_tfw_iteration_converges_to_self_consistent_density():
    w = inputs.small_cell()
    p = scf.Params(lam=0.2, mu=0, history=7, zeta=0.3)
    s = scf.SCF(w.rho, w.b, w.cell.h, w.cell.n_electrons, w.cell.volume, p)
    errs = [s.step() for _ in range(16)]
    assert errs[-1] < 1e-8 and errs[-1] < 1e-6 * errs[0]
    # self-consistency: U(v) at the final v has phi[u] = v
    g, _ = poisson.rhs(s.u * s.u, w.b)
    phi = poisson.solve_exact(g, w.cell.h)
    assert np.linalg.norm(phi - s.v) / np.linalg.norm(s.v) < 1e-7
    r, _ = density.el_residual(s.u, phi, w.cell.h, 0.2, w.cell.n_electrons)
    assert r < 1e-7


def test_anderson_beats_simple_mixing():
    w = inputs.small_cell()
    out = []
    for m in (0, 7):
        p = scf.Params(lam=0.2, mu=0, history=m, zeta=0.3)
        s = scf.SCF(w.rho, w.b, w.cell.h, w.cell.n_electrons, w.cell.volume, p)
        out.append([s.step() for _ in range(8)][-1])
    assert out[1] < 1e-2 * out[0]


def test_update_with_hartree_inside_gives_the_tfw_ground_state():
    """U with the electrostatics inside (the paper's map at mu = 0) reaches in
    one call the density that the potential-mixing iteration converges to
    (separate Poisson solves, Anderson mixing): two routes, one minimiser."""
    w = inputs.small_cell()
    c = w.cell
    u, it, res, _ = density.update(np.sqrt(w.rho), np.zeros(w.rho.shape), c.h, 0.2, c.n_electrons, 6,
                                   tol=1e-11, b=w.b)
    assert res <= 1e-11
    s = scf.SCF(w.rho, w.b, c.h, c.n_electrons, c.volume, scf.Params(lam=0.2, mu=0, history=7, zeta=0.3,
                                                                      u_tol=1e-12))
    for _ in range(40):
        if s.step() < 1e-12:
            break
    assert np.abs(u - s.u).max() <= 1e-8 * np.abs(u).max()
    phi = density.hartree(u, w.b, c.h)
    r, _ = density.el_residual(u, phi, c.h, 0.2, c.n_electrons)
    assert r <= 1e-10
    # the kernel-potential iteration at mu = 0 is that single call
    k = scf.KernelPotentialSCF(w.rho, w.b, c.h, c.n_electrons, c.volume, scf.Params(lam=0.2, mu=0, u_tol=1e-11))
    assert k.step() == 0.0 and np.abs(k.u - u).max() <= 1e-9 * np.abs(u).max()


def test_kernel_potential_fixed_point_converges_to_the_same_ground_state():
    """The paper's fixed point in V_LR (Anderson m = 3, zeta = 1, its Section 5
    settings) on the 4-atom cell with soft (sigma = 1.2) pseudocharges:
    converges below 1e-7, is self-consistent (V = V_LR[u], Euler-Lagrange
    residual of the full H), and lands on the density that the
    potential-mixing iteration reaches from the same start."""
    w = inputs.cubic_workload(1, 16, 1, jitter=0.05, sigma=1.2)
    c = w.cell
    p = scf.Params(lam=1.0, mu=1, history=3, zeta=1.0, u_tol=1e-10)
    k = scf.KernelPotentialSCF(w.rho, w.b, c.h, c.n_electrons, c.volume, p)
    errs = []
    for _ in range(20):
        errs.append(k.step())
        if errs[-1] < 1e-8:
            break
    assert errs[-1] < 1e-8 and len(errs) <= 18, errs
    v_lr = scf.kernel_potential(k.u, c.h, c.n_electrons, c.volume)
    assert np.linalg.norm(v_lr - k.V) / np.linalg.norm(v_lr) < 1e-7
    phi = density.hartree(k.u, w.b, c.h)
    r, _ = density.el_residual(k.u, phi + v_lr, c.h, 1.0, c.n_electrons)
    assert r < 1e-7
    s = scf.SCF(w.rho, w.b, c.h, c.n_electrons, c.volume, scf.Params(lam=1.0, mu=1, history=7, zeta=0.3,
                                                                      u_tol=1e-10))
    for _ in range(40):
        if s.step() < 1e-9:
            break
    assert np.abs(k.u - s.u).max() <= 1e-6 * np.abs(k.u).max()
