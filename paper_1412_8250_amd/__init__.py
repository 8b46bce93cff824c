"""MI355X (gfx950) implementation of the hot path of periodic real-space OF-DFT
with higher-order finite differences (arXiv:1412.8250).

This module only marshals arguments to the C-ABI library ``libofdft.so``
(declared in ``include/ofdft.h``); every step of the computation runs in the
library's HIP kernels.  Tensors are torch CUDA tensors (device memory and
streams only).  The library must be built (``python -m
paper_1412_8250_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libofdft.so")

OK, NOT_CONVERGED, INVALID_ARG, NONFINITE, BREAKDOWN, HIP_ERROR, NO_MEMORY = 0, 1, -1, -2, -3, -4, -5
F64, F32, C128, C64 = 0, 1, 2, 3
PLAIN_F64, REFINED_F32, LEARNED = 0, 1, 2


class OfdftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"status {status}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("nn_applies", ctypes.c_int), ("fell_back", ctypes.c_int),
                ("status", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("removed_mean", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ScfParams(ctypes.Structure):
    _fields_ = [("grid", Grid), ("radius", ctypes.c_int), ("lam", ctypes.c_double),
                ("mu", ctypes.c_int), ("n_electrons", ctypes.c_double), ("history", ctypes.c_int),
                ("zeta", ctypes.c_double), ("u_tol", ctypes.c_double), ("n_restart", ctypes.c_int),
                ("u_max_iter", ctypes.c_int), ("poisson_tol", ctypes.c_double),
                ("poisson_mode", ctypes.c_int), ("helmholtz_tol", ctypes.c_double),
                ("helmholtz_dtype", ctypes.c_int), ("max_iter", ctypes.c_int)]


_lib = None
_V = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_GP = ctypes.POINTER(Grid)
_SP = ctypes.POINTER(SolveStats)


def _declare(l):
    sig = {
        "ofdft_last_error": (_I, [ctypes.c_char_p, ctypes.c_size_t]),
        "ofdft_version": (ctypes.c_char_p, []),
        "fd_laplacian_apply": (_I, [_GP, _I, _I, _V, _V, _D, _D, _V]),
        "ofdft_poisson_create": (_I, [_GP, _I, _I, ctypes.POINTER(_V)]),
        "ofdft_poisson_destroy": (_I, [_V]),
        "cg_poisson_solve": (_I, [_V, _V, _V, _D, _I, _SP, _V]),
        "ofdft_batch_create": (_I, [_I, _GP, _I, _I, ctypes.POINTER(_V)]),
        "ofdft_batch_destroy": (_I, [_V]),
        "cg_helmholtz_solve_batched": (_I, [_V, ctypes.POINTER(_D), ctypes.POINTER(_V),
                                            ctypes.POINTER(_V), _D, _I, _SP, _V]),
        "ofdft_anderson_create": (_I, [ctypes.c_int64, _I, _D, ctypes.POINTER(_V)]),
        "ofdft_anderson_destroy": (_I, [_V]),
        "ofdft_anderson_reset": (_I, [_V]),
        "anderson_mix": (_I, [_V, _V, _V, _V, _V]),
        "ofdft_scf_create": (_I, [ctypes.POINTER(ScfParams), _V, _V, ctypes.POINTER(_V), _V]),
        "ofdft_scf_destroy": (_I, [_V]),
        "ofdft_scf_step": (_I, [_V, ctypes.POINTER(_D), _V]),
        "ofdft_scf_get": (_I, [_V, _I, _V, _V]),
        "ofdft_scf_set": (_I, [_V, _I, _V, _V]),
        "ofdft_scf_stats": (_I, [_V, ctypes.POINTER(_D)]),
        "ofdft_density_update": (_I, [_V, _V, _V, ctypes.POINTER(_I), ctypes.POINTER(_D),
                                      ctypes.POINTER(_D), _V]),
        "ofdft_stencil_set_config": (_I, [_I, _I, _I, _I, _I, _I]),
    }
    for name, (res, args) in sig.items():
        if not hasattr(l, name):
            continue
        f = getattr(l, name)
        f.restype = res
        f.argtypes = args


def lib():
    """Load libofdft.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1412_8250_amd.build`")
        l = ctypes.CDLL(LIB_PATH)
        _declare(l)
        _lib = l
    return _lib


def last_error() -> str:
    buf = ctypes.create_string_buffer(2048)
    lib().ofdft_last_error(buf, len(buf))
    return buf.value.decode()


def _check(status, ok=(OK,)):
    if status not in ok:
        raise OfdftError(status, last_error())
    return status


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def grid_of(shape_zyx: Sequence[int], h_xyz: Sequence[float]) -> Grid:
    nz, ny, nx = shape_zyx
    return Grid(int(nx), int(ny), int(nz), float(h_xyz[0]), float(h_xyz[1]), float(h_xyz[2]))


_DT = {"torch.float64": F64, "torch.float32": F32, "torch.complex128": C128, "torch.complex64": C64}


def _dtype_code(t) -> int:
    code = _DT.get(str(t.dtype))
    if code is None:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return code


def _dev(t, shape=None):
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
def fd_laplacian_apply(x, y, h_xyz, radius: int = 6, alpha: float = 1.0, beta: float = 0.0,
                       stream=None):
    """y = alpha L_h x + beta y (periodic, order 2*radius)."""
    if x.dtype != y.dtype or x.shape != y.shape:
        raise ValueError("x and y must share dtype and shape")
    g = grid_of(x.shape, h_xyz)
    _check(lib().fd_laplacian_apply(ctypes.byref(g), int(radius), _dtype_code(x), _dev(x), _dev(y),
                                    float(alpha), float(beta), _stream(stream)))
    return y


def set_stencil_config(shape_zyx, elem_bytes: int, shape_id: int, zlen: int = 0):
    nz, ny, nx = shape_zyx
    _check(lib().ofdft_stencil_set_config(nx, ny, nz, elem_bytes, shape_id, zlen))


class PoissonSolver:
    """Workspace for -L_h phi = P g on one grid (plain FP64 / refined FP32 / learned)."""

    def __init__(self, shape_zyx, h_xyz, radius: int = 6, mode: int = PLAIN_F64):
        self.shape = tuple(shape_zyx)
        self.grid = grid_of(shape_zyx, h_xyz)
        self._h = ctypes.c_void_p()
        _check(lib().ofdft_poisson_create(ctypes.byref(self.grid), int(radius), int(mode),
                                          ctypes.byref(self._h)))

    def solve(self, rhs, x, rel_tol: float = 1e-10, max_iter: int = 100000, stream=None,
              allow_not_converged: bool = False) -> dict:
        st = SolveStats()
        ok = (OK, NOT_CONVERGED) if allow_not_converged else (OK,)
        status = lib().cg_poisson_solve(self._h, _dev(rhs, self.shape), _dev(x, self.shape),
                                        float(rel_tol), int(max_iter), ctypes.byref(st),
                                        _stream(stream))
        out = st.as_dict()
        out["status"] = status
        _check(status, ok)
        return out

    def close(self):
        if self._h:
            lib().ofdft_poisson_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
