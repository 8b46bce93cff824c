"""Seeded input generators: neutrality, normalisation, determinism."""
import numpy as np

from paper_1412_8250_amd import inputs


def test_small_cell_neutral_and_normalised():
    w = inputs.small_cell()
    dv = np.prod(w.cell.h)
    assert len(w.cell.atoms) == 4
    assert abs(dv * w.b.sum() + 12.0) < 1e-9        # -3 e per atom, images included
    assert abs(dv * (w.rho + w.b).sum()) < 1e-10
    assert w.rho.min() > 0
    rho_bar = 12.0 / 7.5 ** 3
    assert np.abs(w.rho / rho_bar - 1).max() < 0.06


def test_determinism_and_seeds():
    a, b = inputs.small_cell(1), inputs.small_cell(1)
    assert np.array_equal(a.rho, b.rho) and np.array_equal(a.b, b.b)
    c = inputs.small_cell(7)
    assert not np.array_equal(a.rho, c.rho)


def test_vacancy_and_jitter():
    rng = np.random.default_rng(0)
    full = inputs.fcc_atoms((3, 3, 3), 7.5, 0.0, rng)
    vac = inputs.fcc_atoms((3, 3, 3), 7.5, 0.0, rng, vacancy=True)
    assert len(full) == 108 and len(vac) == 107
    jit = inputs.fcc_atoms((3, 3, 3), 7.5, 0.05, np.random.default_rng(1))
    d = jit - full
    d -= 22.5 * np.round(d / 22.5)
    assert 0.03 < d.std() < 0.07


def test_gaussian_pseudocharge_shape():
    cell = inputs.Cell((24, 24, 24), (15.0,) * 3, np.array([[3.0, 4.0, 5.0]]))
    b = inputs.pseudocharge(cell, sigma=0.8)
    dv = np.prod(cell.h)
    assert abs(dv * b.sum() + 3.0) < 1e-10
    k, j, i = np.unravel_index(np.argmin(b), b.shape)
    assert np.allclose(np.array([i, j, k]) * 0.625, [3.0, 4.0, 5.0], atol=0.32)


def test_batched_cell_sizes_and_shifts():
    sizes = inputs.batched_cell_sizes()
    assert len(sizes) == 32
    for m, n in sizes:
        assert n % 8 == 0 and 24 <= n <= 96 and m in (2, 3, 4, 5)
        assert 0.385 <= m * 7.5 / n <= 0.63
    kappa, c = inputs.shifted_system_draws(np.random.default_rng(0), 1000)
    assert (kappa.real > 0).all()
    assert (np.abs(kappa) >= 0.1 - 1e-12).all() and (np.abs(kappa) <= 5 + 1e-12).all()
    assert np.allclose(np.abs(c), 1.0)


def test_device_generator_equals_numpy_recipe():
    """The torch evaluation of the training and held-out cells (run here on
    the CPU) reproduces the numpy recipes: same atoms, same draws, the same
    Gaussians and field up to rounding."""
    import torch
    from paper_1412_8250_amd import inputs
    for i in (0, 3):
        w = inputs.training_workload(i)
        cell, b, rho = inputs.training_cell_torch(i, "cpu")
        assert np.array_equal(cell.atoms, w.cell.atoms)
        assert np.abs(b.numpy() - w.b).max() <= 1e-13 * np.abs(w.b).max()
        assert np.abs(rho.numpy() - w.rho).max() <= 1e-13 * np.abs(w.rho).max()
    w = inputs.heldout_workload(0)
    cell, b, rho = inputs.heldout_cell_torch(0, "cpu")
    assert np.abs(b.numpy() - w.b).max() <= 1e-13 * np.abs(w.b).max()
    assert np.abs(rho.numpy() - w.rho).max() <= 1e-13 * np.abs(w.rho).max()
    del torch
