"""The allocation-free Poisson entry point (cg_poisson_solve_noalloc) against
the context-based cg_poisson_solve of the plain FP64 form: two calls in a
row on the static workspace, the second on a smaller, ragged grid, each equal
to the existing entry point's result and meeting the tolerance by the
oracle's FP64 residual; grids beyond the static workspace are refused."""
import numpy as np
import pytest

import paper_1412_8250_amd as ofd
from oracle import poisson
from paper_1412_8250_amd import inputs
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


def _rhs(shape, h, seed):
    rng = np.random.default_rng(seed)
    g = rng.normal(size=shape)
    return g - g.mean() + 0.1            # a non-neutral right-hand side: its mean is removed


def _both(g, h, tol):
    torch = torch_cuda()
    gd = to_dev(g)
    x_ref = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    s = ofd.PoissonSolver(g.shape, h, 6, ofd.PLAIN_F64)
    st_ref = s.solve(gd, x_ref, tol)
    s.close()
    x = torch.zeros_like(x_ref)
    st = ofd.poisson_solve_noalloc(gd, x, h, tol)
    return to_host(x_ref), st_ref, to_host(x), st


def test_noalloc_poisson_matches_context_solve_twice():
    w = inputs.supercell_500()                       # 96^3, the largest grid size in the workspace
    h = w.cell.h
    g, _ = poisson.rhs(w.rho, w.b)
    for k, (gg, hh, tol) in enumerate(((g, h, 1e-8), (_rhs((40, 36, 34), (0.41, 0.44, 0.47), 5), (0.41, 0.44, 0.47),
                                                        1e-10))):
        announce("no-alloc Poisson call", k, gg.shape, tol)
        x_ref, st_ref, x, st = _both(gg, hh, tol)
        assert st["status"] == ofd.OK and st_ref["status"] == ofd.OK
        # same kernels in the same order: bitwise the existing entry point's result
        assert np.array_equal(x, x_ref), np.abs(x - x_ref).max()
        assert st["iters"] == st_ref["iters"] and st["rel_res"] == st_ref["rel_res"]
        assert abs(st["removed_mean"] - st_ref["removed_mean"]) <= 1e-15 * max(1.0, abs(st_ref["removed_mean"]))
        # and the oracle's FP64 residual meets the tolerance
        assert poisson.residual(x, gg, hh) <= 1.0001 * tol
        assert abs(x.mean()) <= 1e-12 * np.abs(x).max()
