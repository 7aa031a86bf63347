"""The C-ABI library loads and exports every entry point its headers declare (no GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2204_04321_amd", "libfo_stokes.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        for m in re.finditer(r"\b(fo_[a-z0-9_]+)\s*\(", src):
            names.add(m.group(1))
    return sorted(names)


def test_headers_declare_the_core_entry_points():
    names = declared_functions()
    for n in ("fo_mesh_create", "fo_mesh_destroy", "fo_mesh_info", "fo_jacobian_pattern",
              "fo_assemble_residual", "fo_assemble_jacobian", "fo_initial_guess_sia",
              "fo_status_string", "fo_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_status_strings_and_null_checks_without_gpu():
    from paper_2204_04321_amd import _lib
    L = _lib.lib()
    assert L.fo_status_string(0) == b"ok"
    assert L.fo_status_string(-4) == b"degenerate mesh"
    # argument validation happens before any device call
    out = ctypes.c_void_p()
    assert L.fo_mesh_create(None, None, ctypes.byref(out)) == _lib.FO_EINVAL
    assert b"desc is NULL" in L.fo_last_error()
    assert L.fo_mesh_info(None, None, None, None, None) == _lib.FO_EINVAL
    assert L.fo_assemble_residual(None, None, None, None) == _lib.FO_EINVAL
    assert L.fo_assemble_jacobian(None, None, None, None, 0, 0, None) == _lib.FO_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asking for more exits with status 2 and says why."""
    import subprocess
    import sys
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
