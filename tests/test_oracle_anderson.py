"""Pins of the oracle's Anderson mixing (Appendix D)."""
import numpy as np
import pytest

from oracle.anderson import Anderson


def test_no_history_is_simple_mixing():
    rng = np.random.default_rng(0)
    a = Anderson(0, 0.3)
    v = rng.normal(size=50)
    for _ in range(3):
        f = rng.normal(size=50)
        nv = a.step(v, f)
        assert np.allclose(nv, v + 0.3 * f, rtol=0, atol=1e-15)
        v = nv


@pytest.mark.parametrize("d", [1, 3, 5])
def test_finite_termination_on_linear_map(d):
    """For f(v) = c - A v in dimension d <= m, Anderson mixing is equivalent to
    GMRES and reaches the fixed point after at most d + 1 steps."""
    rng = np.random.default_rng(d)
    A = rng.normal(size=(d, d)) * 0.3 + np.eye(d)
    c = rng.normal(size=d)
    vstar = np.linalg.solve(A, c)
    a = Anderson(7, 0.3)
    v = np.zeros(d)
    for k in range(d + 2):
        v = a.step(v, c - A @ v)
    assert np.abs(v - vstar).max() < 1e-10 * max(1.0, np.abs(vstar).max())


def test_scalar_example_by_hand():
    """f(v) = 2 - 4 v, v0 = 0, zeta = 0.5:  v1 = 0 + 0.5*2 = 1;  f1 = -2;
    s = 1, y = -4, gamma = y f1 / y^2 = 0.5;  v2 = 1 + 0.5*(-2) - (1 + 0.5*(-4))*0.5 = 0.5."""
    a = Anderson(3, 0.5)
    v1 = a.step(np.array([0.0]), np.array([2.0]))
    assert v1[0] == 1.0
    v2 = a.step(v1, 2.0 - 4.0 * v1)
    assert abs(v2[0] - 0.5) < 1e-15


def test_rank_deficient_history_drops_oldest():
    a = Anderson(3, 0.3)
    v = np.array([1.0, 2.0, 3.0])
    f = np.array([0.5, 0.5, 0.5])
    for _ in range(4):                 # identical residual differences -> singular Y^T Y
        v2 = a.step(v, f)
        v = v2
        f = f * 1.0
    assert np.all(np.isfinite(v))
