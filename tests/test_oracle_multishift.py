"""Pins of the oracle's multi-shift COCG (shifted systems of one right-hand
side, Section 3.1; the kernel shifts of Appendix A)."""
import numpy as np
import pytest

from oracle import fd, helmholtz, kernel, multishift

SHAPE, H = (8, 9, 10), (0.45, 0.5, 0.41)


def _rhs(seed, shape=SHAPE, real=False):
    rng = np.random.default_rng(seed)
    f = rng.normal(size=shape)
    return f.astype(np.complex128) if real else f + 1j * rng.normal(size=shape)


def _paper_shifts():
    """The four K_00 shifts (2 kF)^2 Q_r of the Al table, for a cell of 4 atoms."""
    return list(kernel.shifts(12.0, 7.5 ** 3)[:4])


@pytest.mark.parametrize("k", [1, 2, 3, 7, 15])
def test_every_shift_follows_its_own_cocg(k):
    """After k steps each shift's iterate is the k-step COCG iterate of its own
    system from zero (shift invariance of the Krylov space)."""
    f = _rhs(1)
    kaps = _paper_shifts() + [0.9 + 0.4j]
    xs, iters, steps = multishift.solve(f, kaps, H, seed=0, tol=0.0, maxit=k)
    assert steps == k and iters == [k] * len(kaps)
    for kap, x in zip(kaps, xs):
        ref, it, _ = helmholtz.solve_cocg(f, kap, H, tol=0.0, maxit=k)
        assert it == k
        assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_converged_shifts_match_spectral_solve(seed):
    f = _rhs(2)
    kaps = _paper_shifts()
    tol = 1e-10
    xs, iters, steps = multishift.solve(f, kaps, H, seed=seed, tol=tol)
    assert max(iters) <= steps
    lam = fd.symbol(SHAPE, H, 6)
    for kap, x in zip(kaps, xs):
        res = helmholtz.residual(x, f, kap, H)
        assert res <= 10 * tol
        exact = helmholtz.solve_exact(f, kap, H)
        inv_norm = 1.0 / np.abs(-lam + kap).min()        # ||A^-1||_2 of the normal matrix A
        err = np.linalg.norm(x - exact)
        assert err <= 1.01 * inv_norm * res * np.linalg.norm(f)


def test_one_shift_is_textbook_cocg():
    f = _rhs(3)
    kap = 0.236 - 0.926j
    xs, iters, steps = multishift.solve(f, [kap], H, tol=1e-11)
    _, it, _ = helmholtz.solve_cocg(f, kap, H, tol=1e-11)
    # the two recurrences round differently: the stopping step may differ by one
    assert iters == [steps] and abs(steps - it) <= 1
    ref, _, _ = helmholtz.solve_cocg(f, kap, H, tol=0.0, maxit=steps)
    assert np.abs(xs[0] - ref).max() <= 1e-10 * np.abs(ref).max()


def test_frozen_shift_keeps_its_iterate():
    """A shift far from the spectrum of -L_h converges first and its iterate is
    the one of the step at which it froze."""
    f = _rhs(4)
    kaps = [-1.68 - 1.66j, 40.0 + 5.0j]
    xs, iters, steps = multishift.solve(f, kaps, H, tol=1e-9)
    assert iters[1] < iters[0] == steps
    ref, it, _ = helmholtz.solve_cocg(f, kaps[1], H, tol=0.0, maxit=iters[1])
    assert np.abs(xs[1] - ref).max() <= 1e-10 * np.abs(ref).max()


def test_conjugate_shifts_of_a_real_rhs_give_conjugate_solutions():
    f = _rhs(5, real=True)
    kaps = _paper_shifts()
    xs, _, _ = multishift.solve(f, kaps, H, seed=0, tol=1e-11)
    assert np.abs(xs[1] - np.conj(xs[0])).max() <= 1e-9 * np.abs(xs[0]).max()
    assert np.abs(xs[3] - np.conj(xs[2])).max() <= 1e-9 * np.abs(xs[2]).max()


def test_zero_rhs():
    xs, iters, steps = multishift.solve(np.zeros(SHAPE, np.complex128), [1.0, 2.0 + 1j], H)
    assert steps == 0 and iters == [0, 0] and all(np.all(x == 0) for x in xs)
