"""Parity of cg_poisson_solve (Section 3.3 Poisson equation; Section 4 zero
mean and warm starts) against the oracle's exact discrete solution.  The
oracle recomputes the true FP64 residual of the GPU's answer with its own
stencil: <= 1e-10 for the FP64 form, <= 1e-8 for the refined form."""
import numpy as np
import pytest

import paper_1412_8250_amd as ofd
from oracle import poisson
from paper_1412_8250_amd import inputs
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _solve(g_np, h, mode, tol, x0=None, max_iter=100000, allow=False):
    torch = torch_cuda()
    s = ofd.PoissonSolver(g_np.shape, h, 6, mode)
    gd = to_dev(g_np)
    xd = to_dev(np.zeros_like(g_np) if x0 is None else x0)
    st = s.solve(gd, xd, tol, max_iter, allow_not_converged=allow)
    return to_host(xd), st


def _check(x, g, h, tol):
    ref = poisson.solve_exact(g - g.mean(), h)
    res = poisson.residual(x, g, h)
    err = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    assert res <= tol, res
    assert abs(x.mean()) <= 1e-12 * np.abs(x).max()
    return err


@pytest.mark.parametrize("mode,tol", [(ofd.PLAIN_F64, 1e-10), (ofd.REFINED_F32, 1e-8)])
def test_small_cell(mode, tol):
    announce("poisson small cell", mode)
    w = inputs.small_cell()
    g, _ = poisson.rhs(w.rho, w.b)
    x, st = _solve(g, w.cell.h, mode, tol)
    err = _check(x, g, w.cell.h, tol)
    assert st["rel_res"] <= tol and st["iters"] > 10
    assert err < 100 * tol


@pytest.mark.parametrize("shape,h", [((18, 20, 22), (0.41, 0.43, 0.45)), ((7, 9, 11), (0.5, 0.6, 0.7)),
                                     ((40, 24, 70), (0.39, 0.4, 0.42))])
@pytest.mark.parametrize("mode,tol", [(ofd.PLAIN_F64, 1e-10), (ofd.REFINED_F32, 1e-8)])
def test_non_cubic_and_ragged(shape, h, mode, tol):
    announce("poisson", shape, mode)
    rng = np.random.default_rng(sum(shape))
    g = rng.normal(size=shape)
    x, st = _solve(g, h, mode, tol)
    _check(x, g, h, tol)
    assert abs(st["removed_mean"] - g.mean()) < 1e-14


@pytest.mark.parametrize("vacancy", [False, True])
@pytest.mark.parametrize("mode,tol", [(ofd.PLAIN_F64, 1e-8), (ofd.REFINED_F32, 1e-8)])
def test_supercell_500(vacancy, mode, tol):
    """5x5x5 FCC cells on 96^3, perfect and with a vacancy."""
    announce("poisson 96^3", vacancy, mode)
    w = inputs.supercell_500(vacancy)
    g, _ = poisson.rhs(w.rho, w.b)
    x, st = _solve(g, w.cell.h, mode, tol)
    err = _check(x, g, w.cell.h, tol)
    assert err < 1e-5


@pytest.mark.parametrize("mode", [ofd.PLAIN_F64, ofd.MULTIGRID])
def test_warm_start_and_projection_and_status(mode):
    """Mean removal, a converged warm start taking no iteration, and the
    iteration cap reported as NOT_CONVERGED after exactly that many
    iterations (plain CG, and the device-driven multigrid CG whose cap falls
    inside a captured block)."""
    torch = torch_cuda()
    announce("poisson warm start", mode)
    w = inputs.small_cell()
    g, _ = poisson.rhs(w.rho, w.b)
    g_off = g + 0.25                                   # non-neutral: mean removed and reported
    x, st = _solve(g_off, w.cell.h, mode, 1e-10)
    assert abs(st["removed_mean"] - 0.25) < 1e-12
    x2, st2 = _solve(g_off, w.cell.h, mode, 1e-10, x0=x)
    assert st2["iters"] == 0 and np.abs(x2 - x).max() < 1e-14
    cap = 3 if mode == ofd.PLAIN_F64 else 2
    x3, st3 = _solve(g, w.cell.h, mode, 1e-10, max_iter=cap, allow=True)
    assert st3["status"] == ofd.NOT_CONVERGED and st3["iters"] == cap and st3["rel_res"] > 1e-10
    assert np.isfinite(x3).all()


def test_uniform_rhs_gives_zero():
    x, st = _solve(np.full((16, 16, 16), 3.0), (0.5,) * 3, ofd.PLAIN_F64, 1e-10)
    assert np.abs(x).max() == 0.0 and st["status"] == 0


def test_nonfinite_rhs_reported():
    torch = torch_cuda()
    g = np.random.default_rng(0).normal(size=(16, 16, 16))
    g[3, 4, 5] = np.nan
    s = ofd.PoissonSolver(g.shape, (0.5,) * 3)
    with pytest.raises(ofd.OfdftError) as e:
        s.solve(to_dev(g), to_dev(np.zeros_like(g)), 1e-10)
    assert e.value.status == ofd.NONFINITE


def test_bitwise_repeatable():
    w = inputs.small_cell()
    g, _ = poisson.rhs(w.rho, w.b)
    a, _ = _solve(g, w.cell.h, ofd.PLAIN_F64, 1e-10)
    b, _ = _solve(g, w.cell.h, ofd.PLAIN_F64, 1e-10)
    assert np.array_equal(a, b)


def test_large_cell_320():
    """16x16x16 FCC cells (16384 atoms) on 320^3: true FP64 residual from the
    oracle's stencil, plain FP64, refined FP32 and multigrid forms, and the
    solution against the oracle's exact DFT-diagonalised solve: the error is
    within ||A^-1|| ||r|| (A = -L_h on the zero-mean space, ||A^-1|| the
    inverse of its smallest non-zero eigenvalue), element by element."""
    from oracle import fd
    announce("poisson 320^3")
    w = inputs.large_cell()
    g, _ = poisson.rhs(w.rho, w.b)
    exact = poisson.solve_exact(g, w.cell.h)
    lam1 = -fd.symbol_1d(w.rho.shape[0], w.cell.h[0], 6)
    inv_norm = 1.0 / lam1[lam1 > 1e-12].min()
    gn = np.linalg.norm(g)
    for mode in (ofd.PLAIN_F64, ofd.REFINED_F32, ofd.MULTIGRID):
        announce("poisson 320^3 mode", mode)
        x, st = _solve(g, w.cell.h, mode, 1e-8)
        res = poisson.residual(x, g, w.cell.h)
        assert res <= 1e-8
        assert abs(x.mean()) <= 1e-12 * np.abs(x).max()
        err = x - exact
        assert np.abs(err).max() <= np.linalg.norm(err) <= 1.01 * inv_norm * res * gn
        announce("max error / max |phi|", float(np.abs(err).max() / np.abs(exact).max()))
        del x, err


@pytest.mark.parametrize("mode", [ofd.PLAIN_F64, ofd.REFINED_F32, ofd.MULTIGRID, ofd.MULTIGRID_F64])
def test_graph_replays_equal_eager(mode):
    """Captured iteration blocks (16 CG iterations; 4 multigrid-preconditioned
    ones, which read the solution array from the device state) replayed with
    host synchronisations in between give bitwise the eager result, on every
    repeat and for every solution array."""
    torch = torch_cuda()
    announce("poisson graphs", mode)
    w = inputs.supercell_500()
    g, _ = poisson.rhs(w.rho, w.b)
    gd = to_dev(g)
    eager = ofd.PoissonSolver(g.shape, w.cell.h, 6, mode)
    eager.set_graphs(False)
    xe = torch.zeros_like(gd)
    ste = eager.solve(gd, xe, 1e-8)
    graphed = ofd.PoissonSolver(g.shape, w.cell.h, 6, mode)
    for rep in range(3):
        xg = torch.zeros_like(gd)
        stg = graphed.solve(gd, xg, 1e-8)
        torch.cuda.synchronize()
        assert stg["iters"] == ste["iters"]
        assert torch.equal(xg, xe), rep
        _ = (xg * 2).sum().item()          # eager work between replays


@pytest.mark.parametrize("mode", [ofd.MULTIGRID, ofd.MULTIGRID_F64])
@pytest.mark.parametrize("which", ["small", "noncubic", "supercell"])
def test_multigrid_form_matches_exact(which, mode):
    """CG preconditioned by the multigrid V-cycle reaches the same solution
    (exact spectral solve of the oracle) in a handful of iterations."""
    torch = torch_cuda()
    announce("poisson multigrid", which, mode)
    if which == "small":
        w = inputs.small_cell()
        g, _ = poisson.rhs(w.rho, w.b)
        h = w.cell.h
    elif which == "noncubic":
        rng = np.random.default_rng(12)
        g = rng.normal(size=(32, 48, 64))
        g -= g.mean()
        h = (0.45, 0.4, 0.5)
    else:
        w = inputs.supercell_500()
        g, _ = poisson.rhs(w.rho, w.b)
        h = w.cell.h
    x, st = _solve(g, h, mode, 1e-10)
    ref = poisson.solve_exact(g, h)
    assert poisson.residual(x, g, h) <= 1e-10
    assert np.abs(x - ref).max() <= 1e-8 * np.abs(ref).max()
    assert st["iters"] <= 25


@pytest.mark.parametrize("mode,tol", [(ofd.MULTIGRID_F64, 1e-12), (ofd.MULTIGRID, 2e-6)])
def test_multigrid_preconditioner_is_symmetric_positive(mode, tol):
    """M = one V-cycle is a fixed symmetric positive definite operator on
    zero-mean vectors: <M a, b> = <a, M b>, <a, M a> > 0, and M is linear
    (to the rounding of the cycle's precision)."""
    torch = torch_cuda()
    announce("multigrid operator", mode)
    shape, h = (48, 32, 64), (0.4, 0.5, 0.45)
    s = ofd.PoissonSolver(shape, h, 6, mode)
    rng = np.random.default_rng(3)
    a = rng.normal(size=shape)
    b = rng.normal(size=shape)
    a -= a.mean()
    b -= b.mean()
    ad, bd = to_dev(a), to_dev(b)
    Ma, Mb, Mab = (torch.empty_like(ad) for _ in range(3))
    s.apply_preconditioner(ad, Ma)
    s.apply_preconditioner(bd, Mb)
    s.apply_preconditioner(2.0 * ad - 3.0 * bd, Mab)
    x1 = float((Ma * bd).sum())
    x2 = float((ad * Mb).sum())
    assert abs(x1 - x2) <= tol * (Ma.norm() * bd.norm()).item()
    assert float((ad * Ma).sum()) > 0 and float((bd * Mb).sum()) > 0
    assert (Mab - (2.0 * Ma - 3.0 * Mb)).abs().max().item() <= tol * Mab.abs().max().item()


@pytest.mark.parametrize("mode,tol", [(ofd.MULTIGRID_F64, 1e-12), (ofd.MULTIGRID, 2e-6)])
def test_multigrid_cycle_matches_reference(mode, tol):
    """The device V-cycle equals the reference cycle value by value."""
    torch = torch_cuda()
    from oracle import multigrid
    for shape, h in (((48, 32, 64), (0.4, 0.5, 0.45)), ((96, 96, 96), (0.390625,) * 3),
                     ((16, 16, 16), (0.47,) * 3)):
        announce("poisson mg cycle", shape, mode)
        s = ofd.PoissonSolver(shape, h, 6, mode)
        rng = np.random.default_rng(6)
        r = rng.normal(size=shape)
        r -= r.mean()
        rd = to_dev(r)
        zd = torch.empty_like(rd)
        s.apply_preconditioner(rd, zd)
        ref = multigrid.vcycle(r, h)
        assert np.abs(to_host(zd) - ref).max() <= tol * np.abs(ref).max()
        s.close()


def test_multigrid_iterations_do_not_grow_with_the_grid():
    torch = torch_cuda()
    its = []
    for n in (32, 64, 128):
        rng = np.random.default_rng(n)
        g = rng.normal(size=(n, n, n))
        g -= g.mean()
        _, st = _solve(g, (12.0 / n,) * 3, ofd.MULTIGRID, 1e-8)
        its.append(st["iters"])
    print("multigrid iterations", its)
    assert max(its) <= 20 and its[-1] <= its[0] + 4


def test_multigrid_rejects_grids_it_cannot_coarsen():
    with pytest.raises(ofd.OfdftError):
        ofd.PoissonSolver((24, 24, 50), (0.4,) * 3, 6, ofd.MULTIGRID)


@pytest.mark.parametrize("which", ["small", "supercell"])
def test_rhs_assembly_matches_oracle(which):
    """g = 4 pi (rho + b) with its mean removed, by the library, against the
    oracle's assembly, and the removed mean."""
    torch_cuda()
    announce("poisson rhs", which)
    w = inputs.small_cell() if which == "small" else inputs.supercell_500()
    ref, mean = poisson.rhs(w.rho, w.b)
    s = ofd.PoissonSolver(w.rho.shape, w.cell.h)
    gd = to_dev(np.zeros_like(w.rho))
    m = s.rhs(to_dev(w.rho), to_dev(w.b), gd)
    g = to_host(gd)
    assert np.abs(g - ref).max() <= 1e-13 * np.abs(ref).max()
    assert abs(m - mean) <= 1e-12 * np.abs(4 * np.pi * (w.rho + w.b)).max()
    assert abs(g.mean()) <= 1e-14 * np.abs(g).max()
    s.close()
