"""The C-ABI library loads and exports every entry point declared in include/*.h
(no GPU needed: nothing here launches work)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, re.M):
            if m.group(1) not in ("if", "while", "for", "sizeof"):
                names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fd_laplacian_apply", "cg_poisson_solve", "cg_helmholtz_solve_batched",
                     "anderson_mix", "ofdft_scf_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_1412_8250_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_version_string():
    from paper_1412_8250_amd import lib
    assert lib().ofdft_version().startswith(b"ofdft-gfx950")


def test_invalid_arguments_are_rejected_without_gpu_work():
    """Argument checks run on the host before anything touches a device."""
    import paper_1412_8250_amd as m
    l = m.lib()
    g = m.Grid(0, 4, 4, 0.5, 0.5, 0.5)
    assert l.fd_laplacian_apply(ctypes.byref(g), 6, m.F64, ctypes.c_void_p(8), ctypes.c_void_p(16),
                                1.0, 0.0, None) == m.INVALID_ARG
    assert "grid sizes" in m.last_error()
    g = m.Grid(4, 4, 4, 0.5, 0.5, 0.5)
    assert l.fd_laplacian_apply(ctypes.byref(g), 7, m.F64, ctypes.c_void_p(8), ctypes.c_void_p(16),
                                1.0, 0.0, None) == m.INVALID_ARG
    assert l.fd_laplacian_apply(ctypes.byref(g), 6, m.F64, None, ctypes.c_void_p(16),
                                1.0, 0.0, None) == m.INVALID_ARG
    g = m.Grid(4, 4, 4, -0.5, 0.5, 0.5)
    assert l.fd_laplacian_apply(ctypes.byref(g), 6, m.F64, ctypes.c_void_p(8), ctypes.c_void_p(16),
                                1.0, 0.0, None) == m.INVALID_ARG
