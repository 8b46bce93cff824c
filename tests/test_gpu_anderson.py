"""Parity of anderson_mix (Appendix D) against the oracle, step by step."""
import numpy as np
import pytest

import paper_1412_8250_amd as ofd
from oracle.anderson import Anderson as OracleAnderson
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,zeta,n", [(0, 0.3, 1000), (3, 1.0, 4096), (7, 0.3, 123457), (8, 0.5, 777)])
def test_matches_oracle_over_steps(m, zeta, n):
    torch = torch_cuda()
    announce("anderson", m, zeta, n)
    rng = np.random.default_rng(m * 100 + n)
    gpu = ofd.Anderson(n, m, zeta)
    orc = OracleAnderson(m, zeta)
    # a nonlinear fixed-point map v -> 0.5 tanh(v) + c on random data
    c = rng.normal(size=n)
    v = rng.normal(size=n)
    vd = to_dev(v)
    for k in range(12):
        f = 0.5 * np.tanh(v) + c - v
        vn_ref = orc.step(v, f)
        fd_ = to_dev(f)
        gpu.mix(vd, fd_)
        vn = to_host(vd)
        assert np.abs(vn - vn_ref).max() <= 1e-9 * max(1.0, np.abs(vn_ref).max()), k
        v = vn_ref
        vd = to_dev(v)


def test_linear_map_terminates():
    torch = torch_cuda()
    d = 5
    rng = np.random.default_rng(3)
    M = rng.normal(size=(d, d)) * 0.3 + np.eye(d)
    c = rng.normal(size=d)
    vstar = np.linalg.solve(M, c)
    gpu = ofd.Anderson(d, 7, 0.3)
    vd = to_dev(np.zeros(d))
    for _ in range(d + 2):
        v = to_host(vd)
        gpu.mix(vd, to_dev(c - M @ v))
    assert np.abs(to_host(vd) - vstar).max() < 1e-9


def test_out_of_place_and_reset():
    torch = torch_cuda()
    n = 100
    v = np.linspace(0, 1, n)
    f = np.cos(v)
    gpu = ofd.Anderson(n, 3, 0.5)
    vd, fd_ = to_dev(v), to_dev(f)
    out = torch.empty_like(vd)
    gpu.mix(vd, fd_, out)
    assert np.allclose(to_host(out), v + 0.5 * f, rtol=0, atol=1e-15)
    assert np.array_equal(to_host(vd), v)
    gpu.reset()
    gpu.mix(vd, fd_, out)
    assert np.allclose(to_host(out), v + 0.5 * f, rtol=0, atol=1e-15)
