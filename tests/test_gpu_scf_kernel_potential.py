"""The paper's own fixed point (Section 3.3: the mixing variable is the kernel
potential V_LR, U holds the electrostatics; fixed_point = 1) against the
oracle: the density update with the electrostatics inside, the TFW ground
state in one step, and the K_00 iteration step by step and at convergence."""
import numpy as np
import pytest

import paper_1412_8250_amd as ofd
from oracle import density, scf
from paper_1412_8250_amd import inputs
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _ctx(w, **kw):
    return ofd.SCF(w.rho.shape, w.cell.h, to_dev(w.b), to_dev(np.sqrt(w.rho)), w.cell.n_electrons,
                   fixed_point=ofd.SCF.KERNEL_POTENTIAL, **kw)


@pytest.mark.parametrize("precond,pmode", [(ofd.PRECOND_NONE, ofd.PLAIN_F64), (ofd.PRECOND_MULTIGRID, ofd.MULTIGRID)])
def test_density_update_with_electrostatics_matches_oracle(precond, pmode):
    """U(0) at lambda = 0.2 with phi re-solved inside: the TFW ground state."""
    torch = torch_cuda()
    announce("density update with electrostatics", precond, pmode)
    w = inputs.small_cell()
    c = w.cell
    ctx = _ctx(w, lam=0.2, u_tol=1e-10, poisson_tol=1e-12, poisson_mode=pmode, u_precond=precond)
    ud = to_dev(np.sqrt(w.rho))
    it, res, eta = ctx.density_update(torch.zeros_like(ud), ud)
    u_ref, it_ref, res_ref, eta_ref = density.update(np.sqrt(w.rho), np.zeros(w.rho.shape), c.h, 0.2,
                                                     c.n_electrons, tol=1e-10, b=w.b)
    u = to_host(ud)
    announce("iterations", it, it_ref, "eta", eta, eta_ref)
    assert res <= 1e-10
    r_orc, _ = density.el_residual(u, density.hartree(u, w.b, c.h), c.h, 0.2, c.n_electrons)
    assert r_orc <= 5e-10                      # the oracle's own check of the GPU answer
    assert abs(eta - eta_ref) < 1e-9
    assert np.abs(u - u_ref).max() < 1e-7 * np.abs(u_ref).max()
    ctx.close()


def test_tfw_step_is_the_ground_state():
    torch = torch_cuda()
    announce("kernel-potential TFW step")
    w = inputs.small_cell()
    c = w.cell
    ctx = _ctx(w, lam=0.2, u_tol=1e-10, poisson_tol=1e-12, poisson_mode=ofd.MULTIGRID,
               u_precond=ofd.PRECOND_MULTIGRID)
    assert ctx.step() == 0.0
    ref = scf.KernelPotentialSCF(w.rho, w.b, c.h, c.n_electrons, c.volume, scf.Params(lam=0.2, mu=0, u_tol=1e-10))
    ref.step()
    ud = torch.empty(w.rho.shape, dtype=torch.float64, device="cuda")
    ctx.get(ofd.SCF.U, ud)
    assert np.abs(to_host(ud) - ref.u).max() < 1e-7 * np.abs(ref.u).max()
    # phi of the context is the field of the final density
    pd = torch.empty_like(ud)
    ctx.get(ofd.SCF.PHI, pd)
    phi = density.hartree(ref.u, w.b, c.h)
    assert np.abs(to_host(pd) - phi).max() < 1e-7 * np.abs(phi).max()
    ctx.close()


def test_kernel_potential_iteration_matches_oracle_and_converges():
    """K_00 (lambda = mu = 1), Anderson m = 3, zeta = 1, the 4-atom cell with
    sigma = 1.2 pseudocharges: residuals step by step, then convergence below
    1e-7 to the oracle's self-consistent density."""
    torch = torch_cuda()
    announce("kernel-potential K_00 iteration")
    w = inputs.cubic_workload(1, 16, 1, jitter=0.05, sigma=1.2)
    c = w.cell
    ctx = _ctx(w, lam=1.0, mu=1, history=3, zeta=1.0, u_tol=1e-10, poisson_tol=1e-12, helmholtz_tol=1e-12,
               poisson_mode=ofd.MULTIGRID, helmholtz_precond=ofd.PRECOND_MULTIGRID, u_precond=ofd.PRECOND_MULTIGRID)
    ref = scf.KernelPotentialSCF(w.rho, w.b, c.h, c.n_electrons, c.volume,
                                 scf.Params(lam=1.0, mu=1, history=3, zeta=1.0, u_tol=1e-10))
    vd = torch.empty(w.rho.shape, dtype=torch.float64, device="cuda")
    ctx.get(ofd.SCF.V, vd)
    assert np.abs(to_host(vd) - ref.V).max() < 1e-8 * np.abs(ref.V).max()
    res_g, res_o = [], []
    for k in range(18):
        res_g.append(ctx.step())
        res_o.append(ref.step())
        announce("step", k, res_g[-1], res_o[-1], ctx.stats())
        if k < 5:
            assert abs(res_g[-1] - res_o[-1]) <= 1e-5 * res_o[-1] + 1e-9, (k, res_g[-1], res_o[-1])
        if res_g[-1] < 1e-8 and res_o[-1] < 1e-8:
            break
    assert res_g[-1] < 1e-7 and len(res_g) <= 18, res_g
    ud = torch.empty_like(vd)
    ctx.get(ofd.SCF.U, ud)
    assert np.abs(to_host(ud) - ref.u).max() < 1e-6 * np.abs(ref.u).max()
    ctx.close()


def test_kernel_potential_checkpoint_refuses_the_other_form(tmp_path):
    torch = torch_cuda()
    w = inputs.small_cell()
    a = _ctx(w, lam=0.2)
    path = str(tmp_path / "k.ck")
    a.save(path)
    b = ofd.SCF(w.rho.shape, w.cell.h, to_dev(w.b), to_dev(np.sqrt(w.rho)), w.cell.n_electrons, lam=0.2)
    with pytest.raises(ofd.OfdftError):
        b.load(path)
    a.close()
    b.close()
