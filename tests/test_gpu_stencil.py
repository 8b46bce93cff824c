"""Parity of fd_laplacian_apply (Section 4, FD Laplacian with periodic images)
against the CPU oracle, element by element, for all four element types."""
import numpy as np
import pytest

from oracle import fd
from tests.gpu_util import announce, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu

SHAPES = [((16, 16, 16), (0.46875,) * 3),
          ((9, 7, 5), (0.31, 0.42, 0.53)),          # smaller than the stencil: repeated wrap
          ((20, 37, 70), (0.4, 0.45, 0.5)),         # ragged tiles in x and y
          ((33, 18, 130), (0.35, 0.39, 0.41)),
          ((96, 96, 96), (0.390625,) * 3),
          ((20, 150, 128), (0.4, 0.45, 0.5))]      # wide: the 64 x 32 tiles of the FP64 apply


def _ref_scale(x, h, N):
    w = np.concatenate([fd.weights(N, hh) for hh in h])
    return np.abs(w).sum() * np.abs(x).max()


@pytest.mark.parametrize("shape,h", SHAPES)
@pytest.mark.parametrize("dtype", ["f64", "f32", "c128", "c64"])
def test_apply_matches_oracle(shape, h, dtype):
    torch = torch_cuda()
    announce("stencil", shape, dtype)
    rng = np.random.default_rng(hash((shape, dtype)) % 2 ** 32)
    x = rng.normal(size=shape)
    if dtype in ("c128", "c64"):
        x = x + 1j * rng.normal(size=shape)
    tdt = {"f64": torch.float64, "f32": torch.float32, "c128": torch.complex128,
           "c64": torch.complex64}[dtype]
    xd = to_dev(x, tdt)
    yd = torch.empty_like(xd)
    from paper_1412_8250_amd import fd_laplacian_apply
    fd_laplacian_apply(xd, yd, h, 6)
    torch.cuda.synchronize()
    # the oracle sees exactly the values the GPU saw (rounded to the input type)
    xin = to_host(xd).astype(np.complex128 if dtype in ("c128", "c64") else np.float64)
    ref = fd.laplacian(xin, h, 6)
    tol = (1e-14 if dtype in ("f64", "c128") else 2e-6) * _ref_scale(xin, h, 6)
    assert np.abs(to_host(yd) - ref).max() <= tol


@pytest.mark.parametrize("dtype", ["f64", "f32", "c128"])
def test_every_launch_shape(dtype):
    """Each tile shape the launch table can hold (set by hand, as the tuner
    does), on a grid with ragged tiles in x and y and short z chunks."""
    torch = torch_cuda()
    import paper_1412_8250_amd as ofd
    shape, h = (26, 70, 136), (0.4, 0.45, 0.5)
    rng = np.random.default_rng(11)
    x = rng.normal(size=shape)
    if dtype == "c128":
        x = x + 1j * rng.normal(size=shape)
    tdt = {"f64": torch.float64, "f32": torch.float32, "c128": torch.complex128}[dtype]
    eb = {"f64": 8, "f32": 4, "c128": 16}[dtype]
    xd = to_dev(x, tdt)
    xin = to_host(xd).astype(np.complex128 if dtype == "c128" else np.float64)
    ref = fd.laplacian(xin, h, 6)
    tol = (1e-14 if dtype != "f32" else 2e-6) * _ref_scale(xin, h, 6)
    try:
        for sid in range(6):
            for zlen in (0, 7):
                announce("stencil shape", dtype, sid, zlen)
                ofd.set_stencil_config(shape, eb, sid, zlen)
                yd = torch.full_like(xd, float("nan"))
                ofd.fd_laplacian_apply(xd, yd, h, 6)
                torch.cuda.synchronize()
                assert np.abs(to_host(yd) - ref).max() <= tol, (sid, zlen)
    finally:
        ofd.set_stencil_config(shape, eb, -1)


@pytest.mark.parametrize("radius", [1, 2, 3, 4, 5, 6])
def test_radius_alpha_beta(radius):
    torch = torch_cuda()
    announce("stencil radius", radius)
    shape, h = (12, 14, 17), (0.3, 0.35, 0.4)
    rng = np.random.default_rng(radius)
    x, y0 = rng.normal(size=(2,) + shape)
    xd, yd = to_dev(x), to_dev(y0)
    from paper_1412_8250_amd import fd_laplacian_apply
    fd_laplacian_apply(xd, yd, h, radius, alpha=-0.7, beta=1.3)
    ref = -0.7 * fd.laplacian(x, h, radius) + 1.3 * y0
    assert np.abs(to_host(yd) - ref).max() <= 1e-14 * _ref_scale(x, h, radius) * 2


def test_beta_zero_ignores_garbage_output():
    torch = torch_cuda()
    shape, h = (16, 16, 16), (0.5,) * 3
    x = np.random.default_rng(0).normal(size=shape)
    xd = to_dev(x)
    yd = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    from paper_1412_8250_amd import fd_laplacian_apply
    fd_laplacian_apply(xd, yd, h, 6)
    assert torch.isfinite(yd).all()


def test_full_size_sampled_and_plane_wave():
    """320^3 (the large-cell grid): sampled points against the oracle's
    point-wise definition, and a plane wave against the exact discrete symbol."""
    torch = torch_cuda()
    announce("stencil 320^3")
    n, h = 320, (0.375,) * 3
    g = torch.Generator(device="cuda").manual_seed(0)
    xd = torch.randn((n, n, n), dtype=torch.float64, device="cuda", generator=g)
    yd = torch.empty_like(xd)
    from paper_1412_8250_amd import fd_laplacian_apply
    fd_laplacian_apply(xd, yd, h, 6)
    rng = np.random.default_rng(1)
    pts = [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(200)]
    pts += [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n - 1, 5), (319, 3, 0)]
    idx = torch.tensor(pts, device="cuda")
    y_s = to_host(yd[idx[:, 0], idx[:, 1], idx[:, 2]])
    # neighbourhoods for the oracle's point-wise evaluation
    x = to_host(xd)
    ref = fd.laplacian_at(x, h, 6, pts)
    assert np.abs(y_s - ref).max() <= 1e-14 * _ref_scale(x, h, 6)
    del x
    k = (3, 7, 11)
    zz, yy, xx = torch.meshgrid(*(torch.arange(n, device="cuda", dtype=torch.float64),) * 3,
                                indexing="ij")
    wave = torch.cos(2 * np.pi * (k[0] * xx + k[1] * yy + k[2] * zz) / n)
    fd_laplacian_apply(wave.contiguous(), yd, h, 6)
    lam = fd.symbol((n, n, n), h, 6)[k[2], k[1], k[0]]
    assert (yd - lam * wave).abs().max().item() <= 1e-13 * abs(fd.symbol((n, n, n), h, 6)).max()
