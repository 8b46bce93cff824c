"""Parity of cocg_multishift_solve (the shifted systems of Section 3.1 that share
one right-hand side; the K_00 shifts of Appendix A) against the oracle's
multi-shift COCG step by step, its spectral solve, and at the benchmark's full
size against the oracle's complex128 residual."""
import numpy as np
import pytest

import paper_1412_8250_amd as ofd
from oracle import fd, helmholtz, kernel, multishift
from paper_1412_8250_amd import inputs
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu

# (shape zyx, h xyz): a 64 x 8 tiled grid with ragged x and y tails and a
# small grid on the 32 x 8 tile
GRIDS = [((20, 26, 70), (0.41, 0.45, 0.38)), ((11, 17, 13), (0.5, 0.44, 0.47))]


def _shifts():
    return list(kernel.shifts(12.0, 7.5 ** 3)[:4]) + [0.9 + 0.4j]


def _run(shape, h, kaps, f, tol, maxit=100000, seed=-1, allow=False):
    torch = torch_cuda()
    ms = ofd.MultiShift(shape, h, 6, max_shifts=len(kaps))
    xs = [torch.full(shape, complex(7.0, -3.0), dtype=torch.complex128, device="cuda") for _ in kaps]
    status, st, used = ms.solve(kaps, to_dev(f.astype(np.complex128)), xs, tol, maxit, seed,
                                allow_not_converged=allow)
    out = [to_host(x) for x in xs]
    ms.close()
    return status, out, st, used


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("steps", [1, 4, 23])
def test_iterates_match_oracle_step_by_step(grid, steps):
    """After a fixed number of steps every shift's iterate equals the oracle's
    (same seed, same recurrences) element by element."""
    shape, h = grid
    announce("multishift steps", shape, steps)
    rng = np.random.default_rng(31)
    f = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    kaps = _shifts()
    status, xs, st, used = _run(shape, h, kaps, f, 1e-300, steps, seed=0, allow=True)
    assert status == ofd.NOT_CONVERGED and used == 0
    ref, iters, k = multishift.solve(f, kaps, h, seed=0, tol=0.0, maxit=steps)
    assert k == steps
    for j, (x, r) in enumerate(zip(xs, ref)):
        assert st[j]["iters"] == steps and st[j]["outer_iters"] == steps
        assert np.abs(x - r).max() <= 1e-11 * np.abs(r).max(), j


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("seed", [-1, 2])
def test_converged_shifts_match_oracle_and_spectral_solve(grid, seed):
    shape, h = grid
    announce("multishift converged", shape, seed)
    rng = np.random.default_rng(32)
    f = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    kaps = _shifts()
    tol = 1e-9
    status, xs, st, used = _run(shape, h, kaps, f, tol, seed=seed)
    assert status == ofd.OK
    # the automatic seed: Re kappa < 0 (a resonance inside the spectrum of -L_h), smallest |Im|
    assert used == (seed if seed >= 0 else 0)
    ref, iters, k = multishift.solve(f, kaps, h, seed=used, tol=tol)
    lam = fd.symbol(shape, h, 6)
    for j, kap in enumerate(kaps):
        res = helmholtz.residual(xs[j], f, kap, h)
        # OK means the true residual meets the tolerance (a shift whose true
        # residual drifted above it got correction solves)
        assert res <= 1.0001 * tol and abs(st[j]["rel_res"] - res) <= 1e-3 * res + 1e-15
        assert st[j]["rel_res"] <= tol
        # the step at which a shift freezes is a threshold decision on COCG's erratic
        # residual: rounding moves it by a few steps (the solutions agree below);
        # correction solves add their steps
        assert iters[j] - 3 <= st[j]["iters"] <= iters[j] + 3 + 30, (j, st[j]["iters"], iters[j])
        exact = helmholtz.solve_exact(f, kap, h)
        inv_norm = 1.0 / np.abs(-lam + kap).min()
        assert np.linalg.norm(xs[j] - exact) <= 1.01 * inv_norm * res * np.linalg.norm(f)
        # both iterations stop at (nearly) the same step: the iterates agree to the tolerance
        assert np.linalg.norm(xs[j] - ref[j]) <= 4 * inv_norm * tol * np.linalg.norm(f)
    # the seed sequence ran until the last shift froze, as the oracle's did
    assert st[0]["outer_iters"] == k and max(s["iters"] for s in st) >= k


def test_one_shift_and_zero_rhs_and_errors():
    torch = torch_cuda()
    shape, h = GRIDS[1]
    announce("multishift edge cases")
    rng = np.random.default_rng(33)
    f = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    kap = 0.236 - 0.926j
    status, xs, st, _ = _run(shape, h, [kap], f, 1e-10)
    assert status == ofd.OK
    assert np.abs(xs[0] - helmholtz.solve_exact(f, kap, h)).max() <= 1e-7 * np.abs(xs[0]).max()
    status, xs, st, _ = _run(shape, h, _shifts(), np.zeros(shape), 1e-8)
    assert status == ofd.OK and all(np.all(x == 0) for x in xs) and all(s["iters"] == 0 for s in st)
    ms = ofd.MultiShift(shape, h, 6, max_shifts=2)
    fd_ = to_dev(f)
    x1 = torch.zeros(shape, dtype=torch.complex128, device="cuda")
    for bad in ([1.0, 2.0, 3.0], [0.0, 1.0]):
        with pytest.raises(ofd.OfdftError):
            ms.solve(bad, fd_, [x1, torch.zeros_like(x1), torch.zeros_like(x1)][:len(bad)], 1e-8)
    with pytest.raises(ofd.OfdftError):
        ms.solve([1.0, 2.0], fd_, [x1, x1], 1e-8)          # the same array twice
    with pytest.raises(ofd.OfdftError):
        ms.solve([1.0], fd_, [fd_], 1e-8)                   # solution aliases the right-hand side
    with pytest.raises(ofd.OfdftError):
        ms.solve([1.0], fd_, [x1], 1e-8, seed=1)
    ms.close()


def test_kernel_shifts_320():
    """The K_00 solves of the large cell (320^3) as two multi-shift solves, one per
    base right-hand side -L_h rho^beta and -L_h rho^alpha, to 1e-8; the oracle's
    C stencil recomputes each whole residual, and conjugate shifts of the real
    right-hand side give conjugate solutions."""
    torch = torch_cuda()
    w = inputs.large_cell()
    h = w.cell.h
    ks = list(kernel.shifts(w.cell.n_electrons, w.cell.volume)[:4])
    ms = ofd.MultiShift(w.rho.shape, h, 6, max_shifts=4)
    for name, a in (("beta", kernel.BETA), ("alpha", kernel.ALPHA)):
        announce("multishift 320^3", name)
        f = -fd.laplacian(w.rho ** a, h)
        xs = [torch.empty(w.rho.shape, dtype=torch.complex128, device="cuda") for _ in ks]
        status, st, used = ms.solve(ks, to_dev(f.astype(np.complex128)), xs, 1e-8)
        assert status == ofd.OK
        u0 = to_host(xs[0])
        for j in range(4):
            assert st[j]["rel_res"] <= 1e-8
            u = u0 if j == 0 else to_host(xs[j])
            assert helmholtz.residual(u, f, ks[j], h) <= 1.05e-8, j
            if j == 1:
                # solves to 1e-8 of conjugate systems agree to about the tolerance
                assert np.linalg.norm(u - np.conj(u0)) <= 1e-6 * np.linalg.norm(u0)
            del u
        del xs, u0, f
    ms.close()


def test_scf_kernel_shifts_match_oracle_table():
    """The shifts and factors an SCF context reports are the oracle's K_00 table
    for its cell (Appendix A, kF of Section 3.1)."""
    torch = torch_cuda()
    announce("scf kernel shifts")
    w = inputs.small_cell()
    scf = ofd.SCF(w.rho.shape, w.cell.h, to_dev(w.b), to_dev(np.sqrt(w.rho)), w.cell.n_electrons,
                  lam=0.2, mu=1)
    ks, ps = scf.kernel_shifts()
    scf.close()
    ref = kernel.shifts(w.cell.n_electrons, w.cell.volume)
    for r in range(4):
        assert abs(ks[r] - ref[r]) <= 1e-12 * abs(ref[r])
        assert ps[r] == kernel.P00[r]


@pytest.mark.parametrize("shape,h,nshift", [((3, 5, 7), (0.5, 0.45, 0.4), 3),      # smaller than the stencil reach
                                            ((9, 12, 66), (0.42, 0.4, 0.37), 16)])  # the maximum shift count
def test_edge_grids_and_maximum_shifts(shape, h, nshift):
    """Every axis shorter than the radius-6 reach (periodic images wrap several
    times), and 16 shifts at once: 9 steps element by element against the oracle."""
    announce("multishift edge", shape, nshift)
    rng = np.random.default_rng(34)
    f = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    mags = np.exp(rng.uniform(np.log(0.2), np.log(6.0), nshift))
    args = rng.uniform(-0.9 * np.pi, 0.9 * np.pi, nshift)
    kaps = [complex(m * np.exp(1j * a)) for m, a in zip(mags, args)]
    status, xs, st, used = _run(shape, h, kaps, f, 1e-300, 9, seed=-1, allow=True)
    ref, _, _ = multishift.solve(f, kaps, h, seed=used, tol=0.0, maxit=9)
    for j, (x, r) in enumerate(zip(xs, ref)):
        assert np.abs(x - r).max() <= 1e-10 * np.abs(r).max(), j


def test_context_reuse_with_fewer_shifts():
    """Two solves in a row on one context (the second with fewer shifts and a
    different right-hand side) give the same results as fresh contexts."""
    torch = torch_cuda()
    shape, h = GRIDS[0]
    announce("multishift reuse")
    rng = np.random.default_rng(35)
    f1 = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    f2 = rng.normal(size=shape) + 0j
    kaps = _shifts()
    ms = ofd.MultiShift(shape, h, 6, max_shifts=5)
    xs = [torch.empty(shape, dtype=torch.complex128, device="cuda") for _ in kaps]
    ms.solve(kaps, to_dev(f1), xs, 1e-9)
    ys = xs[:2]
    _, st, _ = ms.solve(kaps[2:4], to_dev(f2), ys, 1e-9)
    got = [to_host(y) for y in ys]
    ms.close()
    _, fresh, st2, _ = _run(shape, h, kaps[2:4], f2, 1e-9)
    for a, b, s1, s2 in zip(got, fresh, st, st2):
        assert s1["iters"] == s2["iters"]
        assert np.array_equal(a, b)
