"""ctypes loader for the oracle's C part (built by oracle/build.py)."""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        l = ctypes.CDLL(_build.LIB)
        l.orc_fd_weights.argtypes = [_I, _D, _P]
        l.orc_laplacian.argtypes = [_I, _I, _I, _D, _D, _D, _I, _P, _P]
        l.orc_laplacian_z.argtypes = [_I, _I, _I, _D, _D, _D, _I, _P, _P]
        l.orc_cg_poisson.argtypes = [_I, _I, _I, _D, _D, _D, _I, _P, _P, _D, _I, _P]
        l.orc_cg_poisson.restype = _I
        l.orc_cocg.argtypes = [_I, _I, _I, _D, _D, _D, _I, _D, _D, _P, _P, _D, _I, _P]
        l.orc_cocg.restype = _I
        l.orc_threads.restype = _I
        l.orc_set_threads.argtypes = [_I]
        _lib = l
    return _lib


def ptr(a: np.ndarray):
    assert a.flags.c_contiguous and a.dtype in (np.float64, np.complex128)
    return a.ctypes.data_as(_P)
