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


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes mirrors of the parameter structs have the header's size and
    field offsets (compiled with the host C compiler)."""
    import shutil
    import subprocess
    import paper_1412_8250_amd as m
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    checks = {"ofdft_scf_params": m.ScfParams, "ofdft_grid": m.Grid, "ofdft_gauss_atoms": m.GaussAtoms,
              "ofdft_tune_result": m.TuneResult, "ofdft_solve_stats": m.SolveStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ofdft.h"', "int main(void) {"]
    for cname, cls in checks.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            cf = {"lam": "lambda"}.get(fname, fname)
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "abi"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in checks.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_scf_parameters_are_checked_before_gpu_work():
    """An out-of-range line-search slope tolerance (and other bad parameters)
    is rejected by the argument checks, before any device allocation."""
    import paper_1412_8250_amd as m
    l = m.lib()
    p = m.ScfParams()
    p.grid = m.Grid(16, 16, 16, 0.5, 0.5, 0.5)
    p.radius, p.lam, p.mu, p.n_electrons = 6, 0.2, 0, 12.0
    p.history, p.zeta, p.u_tol, p.poisson_tol, p.helmholtz_tol = 7, 0.3, 1e-8, 1e-8, 1e-8
    out = ctypes.c_void_p()
    for field, bad in (("line_slope_tol", 1.0), ("line_slope_tol", -0.1), ("line_slope_tol", float("nan")),
                       ("lr_order", 1), ("u_tol", 0.0)):
        q = m.ScfParams.from_buffer_copy(p)
        setattr(q, field, bad)
        st = l.ofdft_scf_create(ctypes.byref(q), ctypes.c_void_p(8), ctypes.c_void_p(16), ctypes.byref(out), None)
        assert st == m.INVALID_ARG, (field, bad)
        assert "invalid parameters" in m.last_error()
    # the multi-shift switch is 0 or 1
    for extra in ({"helmholtz_multishift": 2}, {"helmholtz_multishift": -1}, {"autotune": 2},
                  {"fixed_point": 2}, {"fixed_point": -1}):
        q = m.ScfParams.from_buffer_copy(p)
        q.mu = 1
        for k, v in extra.items():
            setattr(q, k, v)
        st = l.ofdft_scf_create(ctypes.byref(q), ctypes.c_void_p(8), ctypes.c_void_p(16), ctypes.byref(out), None)
        assert st == m.INVALID_ARG, extra


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU; asking for more exits with a message
    before anything touches a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_noalloc_poisson_refuses_before_gpu_work():
    """The allocation-free Poisson entry point checks its grid against the
    static workspace (2^20 points) and its arguments on the host."""
    import paper_1412_8250_amd as m
    l = m.lib()
    st = m.SolveStats()
    g = m.Grid(128, 128, 65, 0.4, 0.4, 0.4)            # 2^20 + 16384 points
    assert l.cg_poisson_solve_noalloc(ctypes.byref(g), 6, ctypes.c_void_p(256), ctypes.c_void_p(512), 1e-8, 10,
                                      ctypes.byref(st), None) == m.INVALID_ARG
    assert "static workspace" in m.last_error()
    g = m.Grid(16, 16, 16, 0.4, 0.4, 0.4)
    assert l.cg_poisson_solve_noalloc(ctypes.byref(g), 6, ctypes.c_void_p(256), ctypes.c_void_p(256), 1e-8, 10,
                                      ctypes.byref(st), None) == m.INVALID_ARG
    assert l.cg_poisson_solve_noalloc(ctypes.byref(g), 6, ctypes.c_void_p(256), ctypes.c_void_p(512), 0.0, 10,
                                      ctypes.byref(st), None) == m.INVALID_ARG
    assert l.cg_poisson_solve_noalloc(ctypes.byref(g), 7, ctypes.c_void_p(256), ctypes.c_void_p(512), 1e-8, 10,
                                      ctypes.byref(st), None) == m.INVALID_ARG


def test_launch_table_save_and_load(tmp_path):
    """The autotuner's launch table round-trips through its text form (host
    only: no kernel runs), malformed files are refused, and a hand-set entry
    is written with family -1."""
    import paper_1412_8250_amd as m
    m.set_stencil_config((37, 41, 43), 8, 2, 9)
    p1 = tmp_path / "table.txt"
    m.tune_save(str(p1))
    lines = [l.split() for l in p1.read_text().splitlines() if not l.startswith("#")]
    assert ["-1", "43", "41", "37", "8", "2", "9"] in lines
    m.set_stencil_config((37, 41, 43), 8, -1)
    p2 = tmp_path / "table2.txt"
    m.tune_save(str(p2))
    assert ["-1", "43", "41", "37", "8", "2", "9"] not in [l.split() for l in p2.read_text().splitlines()]
    assert m.tune_load(str(p1)) == len(lines)
    m.tune_save(str(p2))
    assert ["-1", "43", "41", "37", "8", "2", "9"] in [l.split() for l in p2.read_text().splitlines()]
    m.set_stencil_config((37, 41, 43), 8, -1)
    bad = tmp_path / "bad.txt"
    bad.write_text("0 10 10 10 8 9 0\n")           # unknown shape id
    with pytest.raises(m.OfdftError):
        m.tune_load(str(bad))
    with pytest.raises(m.OfdftError):
        m.tune_load(str(tmp_path / "missing.txt"))
