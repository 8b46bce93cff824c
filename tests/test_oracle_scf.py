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
