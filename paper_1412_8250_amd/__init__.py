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
PLAIN_F64, REFINED_F32, LEARNED, MULTIGRID, MULTIGRID_F64, LEARNED_REFINED = 0, 1, 2, 3, 4, 5
PRECOND_NONE, PRECOND_MULTIGRID, PRECOND_MULTIGRID_F64 = 0, 1, 2


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
                ("helmholtz_dtype", ctypes.c_int), ("max_iter", ctypes.c_int), ("line_tol", ctypes.c_double),
                ("helmholtz_precond", ctypes.c_int), ("u_precond", ctypes.c_int), ("lr_order", ctypes.c_int),
                ("u_precond_sigma", ctypes.c_double), ("line_slope_tol", ctypes.c_double),
                ("helmholtz_multishift", ctypes.c_int), ("autotune", ctypes.c_int),
                ("fixed_point", ctypes.c_int)]


class TuneResult(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int), ("zlen", ctypes.c_int), ("group", ctypes.c_int),
                ("candidates", ctypes.c_int), ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class GaussAtoms(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int), ("pos", ctypes.POINTER(ctypes.c_double)), ("charge", ctypes.c_double),
                ("sigma", ctypes.c_double), ("cutoff", ctypes.c_double)]


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
        "fd_gradient_apply": (_I, [_GP, _I, _V, _V, _V, _V, _V]),
        "ofdft_poisson_create": (_I, [_GP, _I, _I, ctypes.POINTER(_V)]),
        "ofdft_poisson_destroy": (_I, [_V]),
        "cg_poisson_solve": (_I, [_V, _V, _V, _D, _I, _SP, _V]),
        "cg_poisson_solve_noalloc": (_I, [_GP, _I, _V, _V, _D, _I, _SP, _V]),
        "ofdft_poisson_rhs": (_I, [_V, _V, _V, _V, ctypes.POINTER(_D), _V]),
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
        "ofdft_scf_kernel_shifts": (_I, [_V, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
        "ofdft_scf_reset_history": (_I, [_V]),
        "ofdft_density_update": (_I, [_V, _V, _V, ctypes.POINTER(_I), ctypes.POINTER(_D),
                                      ctypes.POINTER(_D), _V]),
        "ofdft_stencil_set_config": (_I, [_I, _I, _I, _I, _I, _I]),
        "ofdft_batch_set_config": (_I, [_V, _I, _I]),
        "ofdft_batch_set_preconditioner": (_I, [_V, _I]),
        "ofdft_scf_energy": (_I, [_V, ctypes.POINTER(GaussAtoms), ctypes.POINTER(_D), _V]),
        "ofdft_scf_energy_paper_form": (_I, [_V, ctypes.POINTER(GaussAtoms), _D, ctypes.POINTER(_D), _V]),
        "ofdft_scf_forces_paper_form": (_I, [_V, ctypes.POINTER(GaussAtoms), _D, ctypes.POINTER(_D), _V]),
        "ofdft_scf_forces": (_I, [_V, ctypes.POINTER(GaussAtoms), ctypes.POINTER(_D), _V]),
        "ofdft_batch_apply_preconditioner": (_I, [_V, _I, ctypes.POINTER(_D), _V, _V, _V]),
        "ofdft_multishift_create": (_I, [ctypes.POINTER(Grid), _I, _I, ctypes.POINTER(_V)]),
        "ofdft_multishift_destroy": (_I, [_V]),
        "cocg_multishift_solve": (_I, [_V, _I, ctypes.POINTER(_D), _I, _V, ctypes.POINTER(_V), _D, _I,
                                       _SP, ctypes.POINTER(_I), _V]),
        "ofdft_nn_create": (_I, [ctypes.c_uint64, ctypes.POINTER(_V)]),
        "ofdft_nn_destroy": (_I, [_V]),
        "ofdft_nn_param_count": (ctypes.c_size_t, []),
        "ofdft_nn_set_weights": (_I, [_V, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t]),
        "ofdft_nn_get_weights": (_I, [_V, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t, _I]),
        "ofdft_nn_reserve": (_I, [_V, _GP]),
        "ofdft_nn_forward": (_I, [_V, _GP, _V, _V, _D, _V]),
        "ofdft_nn_gradients": (_I, [_V, _GP, _V, _V, ctypes.POINTER(_D), _V]),
        "ofdft_nn_train_step": (_I, [_V, _GP, _V, _V, _D, ctypes.POINTER(_D), _V]),
        "ofdft_poisson_set_network": (_I, [_V, _V]),
        "ofdft_poisson_set_graphs": (_I, [_V, _I]),
        "ofdft_poisson_set_refinement": (_I, [_V, _D, _D]),
        "ofdft_poisson_set_learned_mode": (_I, [_V, _I]),
        "ofdft_poisson_apply_preconditioner": (_I, [_V, _V, _V, _V]),
        "ofdft_nn_set_loss": (_I, [_V, _I]),
        "ofdft_nn_set_precision": (_I, [_V, _I]),
        "ofdft_nn_save": (_I, [_V, ctypes.c_char_p]),
        "ofdft_nn_load": (_I, [_V, ctypes.c_char_p]),
        "ofdft_scf_save": (_I, [_V, ctypes.c_char_p, _V]),
        "ofdft_scf_load": (_I, [_V, ctypes.c_char_p, _V]),
        "ofdft_profile_reset": (_I, [ctypes.c_uint]),
        "ofdft_tune_stencil": (_I, [_GP, _I, _I, _I, _I, ctypes.POINTER(TuneResult), _V]),
        "ofdft_batch_tune": (_I, [_V, ctypes.POINTER(_D), ctypes.POINTER(_V), ctypes.POINTER(_V), _I,
                                  ctypes.POINTER(TuneResult), _V]),
        "ofdft_tune_save": (_I, [ctypes.c_char_p]),
        "ofdft_tune_load": (_I, [ctypes.c_char_p, ctypes.POINTER(_I)]),
        "ofdft_profile_read": (_I, [_I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_D),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_D)]),
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


def fd_gradient_apply(x, gx, gy, gz, h_xyz, radius: int = 6, stream=None):
    """(gx, gy, gz) = FD gradient of x (FP64, periodic, order 2*radius)."""
    for t in (gx, gy, gz):
        if t.dtype != x.dtype or t.shape != x.shape:
            raise ValueError("gradient outputs must match x in dtype and shape")
    g = grid_of(x.shape, h_xyz)
    _check(lib().fd_gradient_apply(ctypes.byref(g), int(radius), _dev(x), _dev(gx), _dev(gy), _dev(gz),
                                   _stream(stream)))
    return gx, gy, gz


KERNEL_CLASSES = ("apply", "cg_stencil", "cg_update", "residual", "cocg", "u_stencil", "u_vector",
                  "anderson", "pointwise", "nn", "cocg_update",
                  "multigrid", "multigrid_c", "ms_stencil", "ms_update")


def profile_reset(timed=()):
    """Clear the launch counters; launches of the named classes get HIP-event timing."""
    mask = 0
    for name in timed:
        mask |= 1 << KERNEL_CLASSES.index(name)
    _check(lib().ofdft_profile_reset(mask))


def profile_read() -> dict:
    """{class: {launches, bytes, timed, ms}} accumulated since the last reset."""
    out = {}
    for k, name in enumerate(KERNEL_CLASSES):
        la, tm = ctypes.c_int64(), ctypes.c_int64()
        by, ms = ctypes.c_double(), ctypes.c_double()
        _check(lib().ofdft_profile_read(k, ctypes.byref(la), ctypes.byref(by), ctypes.byref(tm),
                                        ctypes.byref(ms)))
        out[name] = {"launches": la.value, "bytes": by.value, "timed": tm.value, "ms": ms.value}
    return out


def set_stencil_config(shape_zyx, elem_bytes: int, shape_id: int, zlen: int = 0):
    nz, ny, nx = shape_zyx
    _check(lib().ofdft_stencil_set_config(nx, ny, nz, elem_bytes, shape_id, zlen))


TUNE_APPLY, TUNE_PASS = 0, 1
SHAPE_NAMES = ("64x16/256", "64x8/256", "32x16/256", "64x16/512", "64x8/512", "64x32/512")


def tune_stencil(shape_zyx, h_xyz, dtype: int = F64, family: int = TUNE_APPLY, reps: int = 5,
                 radius: int = 6, stream=None) -> dict:
    """Time every legal launch shape / z chunk of one kernel family on the grid
    and record the fastest (see ofdft_tune_stencil)."""
    g = grid_of(shape_zyx, h_xyz)
    r = TuneResult()
    _check(lib().ofdft_tune_stencil(ctypes.byref(g), int(radius), int(dtype), int(family), int(reps),
                                    ctypes.byref(r), _stream(stream)))
    return r.as_dict()


def tune_save(path: str):
    _check(lib().ofdft_tune_save(str(path).encode()))


def tune_load(path: str) -> int:
    n = ctypes.c_int()
    _check(lib().ofdft_tune_load(str(path).encode(), ctypes.byref(n)))
    return n.value


def poisson_solve_noalloc(rhs, x, h_xyz, rel_tol: float = 1e-10, max_iter: int = 100000, radius: int = 6,
                          stream=None, allow_not_converged: bool = False) -> dict:
    """Plain FP64 Poisson solve on the library's static workspace (no
    allocation; grids up to 2^20 points; calls on one GPU must not overlap)."""
    g = grid_of(x.shape, h_xyz)
    st = SolveStats()
    status = lib().cg_poisson_solve_noalloc(ctypes.byref(g), int(radius), _dev(rhs, x.shape), _dev(x),
                                            float(rel_tol), int(max_iter), ctypes.byref(st), _stream(stream))
    out = st.as_dict()
    out["status"] = status
    _check(status, (OK, NOT_CONVERGED) if allow_not_converged else (OK,))
    return out


class PoissonSolver:
    """Workspace for -L_h phi = P g on one grid (plain FP64 / refined FP32 / learned)."""

    def __init__(self, shape_zyx, h_xyz, radius: int = 6, mode: int = PLAIN_F64):
        self.shape = tuple(shape_zyx)
        self.grid = grid_of(shape_zyx, h_xyz)
        self._h = ctypes.c_void_p()
        _check(lib().ofdft_poisson_create(ctypes.byref(self.grid), int(radius), int(mode),
                                          ctypes.byref(self._h)))

    def rhs(self, rho, b, g, stream=None) -> float:
        """g = 4 pi (rho + b) projected to zero mean (FP64 arrays of the grid);
        returns the removed mean."""
        m = ctypes.c_double()
        _check(lib().ofdft_poisson_rhs(self._h, _dev(rho, self.shape), _dev(b, self.shape), _dev(g, self.shape),
                                       ctypes.byref(m), _stream(stream)))
        return m.value

    def set_refinement(self, inner_min: float, inner_max: float):
        _check(lib().ofdft_poisson_set_refinement(self._h, float(inner_min), float(inner_max)))

    def set_graphs(self, enable: bool):
        _check(lib().ofdft_poisson_set_graphs(self._h, 1 if enable else 0))

    def set_network(self, net):
        """Attach a Network (learned mode only); the solver keeps a reference."""
        self._net = net
        _check(lib().ofdft_poisson_set_network(self._h, net._h if net is not None else None))

    def apply_preconditioner(self, r, z, stream=None):
        """z = M r (multigrid solvers only)."""
        _check(lib().ofdft_poisson_apply_preconditioner(self._h, _dev(r, self.shape), _dev(z, self.shape),
                                                        _stream(stream)))
        return z

    def set_learned_mode(self, precondition: bool):
        """Learned form after the network's starting correction: plain CG
        (False, default) or network-preconditioned flexible CG (True)."""
        _check(lib().ofdft_poisson_set_learned_mode(self._h, 1 if precondition else 0))

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


class HelmholtzBatch:
    """Workspace for many complex shifted systems (-L_h + kappa_j) u_j = f_j."""

    def __init__(self, shapes_zyx, hs_xyz, radius: int = 6, dtype: int = C128):
        self.shapes = [tuple(s) for s in shapes_zyx]
        self.n = len(self.shapes)
        grids = (Grid * self.n)(*[grid_of(s, h) for s, h in zip(self.shapes, hs_xyz)])
        self._grids = grids
        self._h = ctypes.c_void_p()
        _check(lib().ofdft_batch_create(self.n, grids, int(radius), int(dtype), ctypes.byref(self._h)))

    def set_config(self, shape_id: int, group: int):
        _check(lib().ofdft_batch_set_config(self._h, int(shape_id), int(group)))

    def set_preconditioner(self, kind: int):
        """PRECOND_NONE or PRECOND_MULTIGRID (complex128, stepped schedule)."""
        _check(lib().ofdft_batch_set_preconditioner(self._h, int(kind)))

    def apply_preconditioner(self, j: int, kappa, r, z, stream=None):
        """z = M_j r (complex128 tensors of system j's grid) for shift kappa."""
        k = (ctypes.c_double * 2)(float(complex(kappa).real), float(complex(kappa).imag))
        for t in (r, z):
            if str(t.dtype) != "torch.complex128":
                raise TypeError("the preconditioner takes complex128 arrays")
        _check(lib().ofdft_batch_apply_preconditioner(self._h, int(j), k, _dev(r, self.shapes[j]),
                                                      _dev(z, self.shapes[j]), _stream(stream)))
        return z

    def _marshal(self, kappas, rhs, xs):
        if len(kappas) != self.n or len(rhs) != self.n or len(xs) != self.n:
            raise ValueError("one kappa, rhs and x per system")
        k = (ctypes.c_double * (2 * self.n))()
        for j, kj in enumerate(kappas):
            k[2 * j], k[2 * j + 1] = float(complex(kj).real), float(complex(kj).imag)
        for t, s in zip(list(rhs) + list(xs), self.shapes * 2):
            if str(t.dtype) != "torch.complex128":
                raise TypeError("shifted systems take complex128 arrays")
            _dev(t, s)
        fp = (ctypes.c_void_p * self.n)(*[t.data_ptr() for t in rhs])
        xp = (ctypes.c_void_p * self.n)(*[t.data_ptr() for t in xs])
        return k, fp, xp

    def tune(self, kappas, rhs, xs, iters: int = 8, stream=None) -> dict:
        """Time the schedules and tile shapes on these systems (x read only) and
        keep the fastest (see ofdft_batch_tune)."""
        k, fp, xp = self._marshal(kappas, rhs, xs)
        r = TuneResult()
        _check(lib().ofdft_batch_tune(self._h, k, fp, xp, int(iters), ctypes.byref(r), _stream(stream)))
        return r.as_dict()

    def solve(self, kappas, rhs, xs, rel_tol: float = 1e-8, max_iter: int = 100000, stream=None,
              allow_not_converged: bool = False):
        """kappas: sequence of complex; rhs, xs: complex128 CUDA tensors (x = guess in, solution out)."""
        k, fp, xp = self._marshal(kappas, rhs, xs)
        st = (SolveStats * self.n)()
        status = lib().cg_helmholtz_solve_batched(self._h, k, fp, xp, float(rel_tol), int(max_iter),
                                                  st, _stream(stream))
        ok = (OK, NOT_CONVERGED) if allow_not_converged else (OK,)
        _check(status, ok)
        return status, [s.as_dict() for s in st]

    def close(self):
        if self._h:
            lib().ofdft_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MultiShift:
    """Multi-shift COCG: (-L_h + kappa_r) u_r = f for several shifts of one f,
    one Krylov sequence (one stencil per iteration) for all of them."""

    def __init__(self, shape_zyx, h_xyz, radius: int = 6, max_shifts: int = 4):
        self.shape = tuple(shape_zyx)
        self.max_shifts = int(max_shifts)
        self._grid = grid_of(self.shape, h_xyz)
        self._h = ctypes.c_void_p()
        _check(lib().ofdft_multishift_create(ctypes.byref(self._grid), int(radius), self.max_shifts,
                                             ctypes.byref(self._h)))

    def solve(self, kappas, rhs, xs, rel_tol: float = 1e-8, max_iter: int = 100000, seed: int = -1,
              stream=None, allow_not_converged: bool = False):
        """kappas: sequence of complex; rhs and xs: complex128 CUDA tensors of the grid
        (xs overwritten with the solutions).  Returns (status, stats per shift, seed used)."""
        S = len(kappas)
        if len(xs) != S:
            raise ValueError("one solution array per shift")
        for t in [rhs, *xs]:
            if str(t.dtype) != "torch.complex128":
                raise TypeError("multi-shift COCG takes complex128 arrays")
            _dev(t, self.shape)
        k = (ctypes.c_double * (2 * S))()
        for j, kj in enumerate(kappas):
            k[2 * j], k[2 * j + 1] = float(complex(kj).real), float(complex(kj).imag)
        xp = (ctypes.c_void_p * S)(*[t.data_ptr() for t in xs])
        st = (SolveStats * S)()
        used = ctypes.c_int(-1)
        status = lib().cocg_multishift_solve(self._h, S, k, int(seed), _dev(rhs, self.shape), xp,
                                             float(rel_tol), int(max_iter), st, ctypes.byref(used),
                                             _stream(stream))
        ok = (OK, NOT_CONVERGED) if allow_not_converged else (OK,)
        _check(status, ok)
        return status, [s.as_dict() for s in st], used.value

    def close(self):
        if self._h:
            lib().ofdft_multishift_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Anderson:
    """Anderson mixing state (history m, parameter zeta) for vectors of n values."""

    def __init__(self, n: int, m: int, zeta: float):
        self._h = ctypes.c_void_p()
        _check(lib().ofdft_anderson_create(int(n), int(m), float(zeta), ctypes.byref(self._h)))

    def mix(self, v, f, out=None, stream=None):
        out = v if out is None else out
        _check(lib().anderson_mix(self._h, _dev(v), _dev(f), _dev(out), _stream(stream)))
        return out

    def reset(self):
        _check(lib().ofdft_anderson_reset(self._h))

    def close(self):
        if self._h:
            lib().ofdft_anderson_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SCF:
    """Fixed-point iteration context: mixing variable v = phi + mu V_LR
    (fixed_point 0) or the kernel potential V_LR with the electrostatics
    inside U (fixed_point 1, the paper's form)."""

    POTENTIAL, KERNEL_POTENTIAL = 0, 1

    V, U, PHI, VLR = 0, 1, 2, 3

    def __init__(self, shape_zyx, h_xyz, b, u0, n_electrons: float, lam: float = 0.2, mu: int = 0,
                 history: int = 7, zeta: float = 0.3, u_tol: float = 1e-10, n_restart: int = 50,
                 u_max_iter: int = 20000, poisson_tol: float = 1e-10, poisson_mode: int = PLAIN_F64,
                 helmholtz_tol: float = 1e-10, helmholtz_dtype: int = C128, max_iter: int = 100000,
                 radius: int = 6, line_tol: float = 0.0, helmholtz_precond: int = PRECOND_NONE,
                 u_precond: int = PRECOND_NONE, lr_order: int = 0, u_precond_sigma: float = 0.0,
                 line_slope_tol: float = 0.0, helmholtz_multishift: bool = False, stream=None,
                 allow_not_converged: bool = False, autotune: bool = False, fixed_point: int = 0):
        self.shape = tuple(shape_zyx)
        p = ScfParams()
        p.grid = grid_of(shape_zyx, h_xyz)
        p.radius, p.lam, p.mu, p.n_electrons = int(radius), float(lam), int(mu), float(n_electrons)
        p.history, p.zeta, p.u_tol, p.n_restart = int(history), float(zeta), float(u_tol), int(n_restart)
        p.u_max_iter, p.poisson_tol, p.poisson_mode = int(u_max_iter), float(poisson_tol), int(poisson_mode)
        p.helmholtz_tol, p.helmholtz_dtype, p.max_iter = float(helmholtz_tol), int(helmholtz_dtype), int(max_iter)
        p.line_tol = float(line_tol)
        p.helmholtz_precond = int(helmholtz_precond)
        p.u_precond = int(u_precond)
        p.lr_order = int(lr_order)
        p.u_precond_sigma = float(u_precond_sigma)
        p.line_slope_tol = float(line_slope_tol)
        p.helmholtz_multishift = int(bool(helmholtz_multishift))
        p.autotune = int(bool(autotune))
        p.fixed_point = int(fixed_point)
        self.params = p
        self._h = ctypes.c_void_p()
        st = lib().ofdft_scf_create(ctypes.byref(p), _dev(b, self.shape), _dev(u0, self.shape),
                                    ctypes.byref(self._h), _stream(stream))
        _check(st, (OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        self.status = st

    def step(self, stream=None, allow_not_converged: bool = False) -> float:
        """One fixed-point step; returns ||vhat - v|| / ||v||.  self.status holds
        the call's status (NOT_CONVERGED if U(v) or a solve missed its tolerance,
        accepted only with allow_not_converged)."""
        res = ctypes.c_double()
        st = lib().ofdft_scf_step(self._h, ctypes.byref(res), _stream(stream))
        _check(st, (OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        self.status = st
        return res.value

    def get(self, which: int, out, stream=None):
        """Copy state vector `which` into `out` (float64 for 0..3, complex128 for the
        shifted-system solutions 4..11 (lr_order 0) or 4..35 (lr_order 2))."""
        _check(lib().ofdft_scf_get(self._h, int(which), _dev(out, self.shape), _stream(stream)))
        return out

    def set(self, which: int, src, stream=None):
        _check(lib().ofdft_scf_set(self._h, int(which), _dev(src, self.shape), _stream(stream)))

    def reset_history(self):
        _check(lib().ofdft_scf_reset_history(self._h))

    def save(self, path: str, stream=None):
        """Checkpoint the iteration state (arrays, Anderson history, line-search memory) to a file."""
        _check(lib().ofdft_scf_save(self._h, str(path).encode(), _stream(stream)))

    def load(self, path: str, stream=None):
        """Resume from a checkpoint written by save() of a context with the same settings."""
        _check(lib().ofdft_scf_load(self._h, str(path).encode(), _stream(stream)))

    def snapshot(self):
        """Device copies of every state vector (restorable with restore())."""
        import torch
        snap = {}
        nsol = (8 if self.params.lr_order == 0 else 32) if self.params.mu else 0
        for which in range(4 + nsol):
            dt = torch.float64 if which < 4 else torch.complex128
            t = torch.empty(self.shape, dtype=dt, device="cuda")
            self.get(which, t)
            snap[which] = t
        return snap

    def restore(self, snap):
        for which, t in snap.items():
            self.set(which, t)
        self.reset_history()

    def kernel_shifts(self):
        """The four K_00 shifts kappa_r and factors P_r of this cell (lists of complex)."""
        k, f = (ctypes.c_double * 8)(), (ctypes.c_double * 8)()
        _check(lib().ofdft_scf_kernel_shifts(self._h, k, f))
        return ([complex(k[2 * r], k[2 * r + 1]) for r in range(4)],
                [complex(f[2 * r], f[2 * r + 1]) for r in range(4)])

    def stats(self) -> dict:
        out = (ctypes.c_double * 7)()
        _check(lib().ofdft_scf_stats(self._h, out))
        keys = ("u_iters", "poisson_iters", "helmholtz_iters", "u_res", "poisson_res",
                "helmholtz_res", "eta")
        return dict(zip(keys, list(out)))

    ENERGY_TERMS = ("tf", "vw", "xc", "electrostatic", "self", "overlap", "kernel", "total")

    @staticmethod
    def _atoms(pos, charge, sigma, cutoff):
        import numpy as _np
        p = _np.ascontiguousarray(_np.asarray(pos, dtype=_np.float64).reshape(-1, 3))
        a = GaussAtoms(len(p), p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(charge), float(sigma),
                       float(8.5 * sigma if cutoff is None else cutoff))
        return a, p

    def energy(self, pos, charge: float = -3.0, sigma: float = 0.8, cutoff=None, stream=None) -> dict:
        """Energy terms (hartree) of the current state for Gaussian pseudocharges at pos (M x 3, bohr)."""
        a, keep = self._atoms(pos, charge, sigma, cutoff)
        out = (ctypes.c_double * 8)()
        _check(lib().ofdft_scf_energy(self._h, ctypes.byref(a), out, _stream(stream)))
        return dict(zip(self.ENERGY_TERMS, list(out)))

    def energy_paper_form(self, pos, sigma_ref: float, charge: float = -3.0, sigma: float = 0.8, cutoff=None,
                          stream=None, allow_not_converged: bool = False) -> dict:
        """Energy terms with the FD-gradient von Weizsacker term and the Appendix B
        grid-form overlap correction (reference Gaussians of width sigma_ref)."""
        a, keep = self._atoms(pos, charge, sigma, 8.5 * max(sigma, sigma_ref) if cutoff is None else cutoff)
        out = (ctypes.c_double * 8)()
        st = lib().ofdft_scf_energy_paper_form(self._h, ctypes.byref(a), float(sigma_ref), out, _stream(stream))
        _check(st, (OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        return dict(zip(self.ENERGY_TERMS, list(out)))

    def forces_paper_form(self, pos, sigma_ref: float, charge: float = -3.0, sigma: float = 0.8, cutoff=None,
                          stream=None, allow_not_converged: bool = False):
        """Forces with the Appendix B grid-form correction (M x 3, hartree/bohr)."""
        import numpy as _np
        a, keep = self._atoms(pos, charge, sigma, 8.5 * max(sigma, sigma_ref) if cutoff is None else cutoff)
        out = _np.zeros((a.count, 3))
        st = lib().ofdft_scf_forces_paper_form(self._h, ctypes.byref(a), float(sigma_ref),
                                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(stream))
        _check(st, (OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        return out

    def forces(self, pos, charge: float = -3.0, sigma: float = 0.8, cutoff=None, stream=None):
        """Forces on the nuclei (M x 3, hartree/bohr) from the current state."""
        import numpy as _np
        a, keep = self._atoms(pos, charge, sigma, cutoff)
        out = _np.zeros((a.count, 3))
        _check(lib().ofdft_scf_forces(self._h, ctypes.byref(a), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      _stream(stream)))
        return out

    def density_update(self, v, u, stream=None, allow_not_converged=False):
        it, res, eta = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
        st = lib().ofdft_density_update(self._h, _dev(v, self.shape), _dev(u, self.shape),
                                        ctypes.byref(it), ctypes.byref(res), ctypes.byref(eta),
                                        _stream(stream))
        _check(st, (OK, NOT_CONVERGED) if allow_not_converged else (OK,))
        return it.value, res.value, eta.value

    def close(self):
        if self._h:
            lib().ofdft_scf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


NN_LAYERS = (("c0a", 1, 16), ("c0b", 16, 16), ("c1a", 16, 32), ("c1b", 32, 32), ("c2a", 32, 64),
             ("c2b", 64, 64), ("c3a", 64, 64), ("c3b", 64, 64), ("d2a", 128, 64), ("d2b", 64, 64),
             ("d1a", 96, 32), ("d1b", 32, 32), ("d0a", 48, 16), ("d0b", 16, 16), ("out", 16, 1))


class Network:
    """The learned solver aid's U-Net (weights on the GPU; see include/ofdft.h)."""

    def __init__(self, seed: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().ofdft_nn_create(int(seed), ctypes.byref(self._h)))
        self.count = int(lib().ofdft_nn_param_count())

    def _flat(self, layers):
        import numpy as np
        return np.ascontiguousarray(np.concatenate(
            [np.asarray(layers[name], dtype=np.float32).reshape(-1) for name, _, _ in NN_LAYERS]))

    def _split(self, flat):
        out, off = {}, 0
        for name, ci, co in NN_LAYERS:
            k = 27 * ci * co
            out[name] = flat[off:off + k].reshape(27, ci, co)
            off += k
        return out

    def set_weights(self, layers):
        flat = self._flat(layers)
        _check(lib().ofdft_nn_set_weights(self._h, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          flat.size))

    def get_weights(self, gradients: bool = False):
        import numpy as np
        flat = np.empty(self.count, dtype=np.float32)
        _check(lib().ofdft_nn_get_weights(self._h, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          flat.size, 1 if gradients else 0))
        return self._split(flat)

    def forward(self, x, out, h_xyz, scale: float = 1.0, stream=None):
        g = grid_of(x.shape, h_xyz)
        _check(lib().ofdft_nn_forward(self._h, ctypes.byref(g), _dev(x), _dev(out, x.shape),
                                      float(scale), _stream(stream)))
        return out

    L2, ENERGY, RESIDUAL = 0, 1, 2

    def set_loss(self, kind: int):
        """Training loss: Network.L2 (solution error), Network.ENERGY (A-norm
        error) or Network.RESIDUAL (norm of the residual the output leaves)."""
        _check(lib().ofdft_nn_set_loss(self._h, int(kind)))

    def save(self, path: str):
        """Checkpoint weights, Adam moments and step count to a file."""
        _check(lib().ofdft_nn_save(self._h, str(path).encode()))

    def load(self, path: str):
        """Resume from a checkpoint written by save()."""
        _check(lib().ofdft_nn_load(self._h, str(path).encode()))

    def set_precision(self, fp32: bool):
        """Activation storage of the kernels: BF16 (default) or FP32 (the FP32
        mode of the same kernels)."""
        _check(lib().ofdft_nn_set_precision(self._h, 1 if fp32 else 0))

    def gradients(self, g_rhs, phi, h_xyz, stream=None) -> float:
        g = grid_of(g_rhs.shape, h_xyz)
        loss = ctypes.c_double()
        _check(lib().ofdft_nn_gradients(self._h, ctypes.byref(g), _dev(g_rhs), _dev(phi, g_rhs.shape),
                                        ctypes.byref(loss), _stream(stream)))
        return loss.value

    def train_step(self, g_rhs, phi, h_xyz, lr: float, stream=None) -> float:
        g = grid_of(g_rhs.shape, h_xyz)
        loss = ctypes.c_double()
        _check(lib().ofdft_nn_train_step(self._h, ctypes.byref(g), _dev(g_rhs), _dev(phi, g_rhs.shape),
                                         float(lr), ctypes.byref(loss), _stream(stream)))
        return loss.value

    def close(self):
        if self._h:
            lib().ofdft_nn_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
