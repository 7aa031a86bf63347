"""The C-ABI library loads and exports every entry point its headers declare (no GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2204_04321_amd", "libfo_stokes.so")
PROBE_LIB = os.path.join(ROOT, "paper_2204_04321_amd", "libfo_probe.so")
# each header's entry points live in one library: the device probes in their own
LIB_OF_HEADER = {"fo_probe.h": PROBE_LIB}


def declared_functions(headers=None):
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        if headers is not None and os.path.basename(h) not in headers:
            continue
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
              "fo_newton_solve", "fo_initial_guess_learned", "fo_learned_targets", "fo_feature_stats",
              "fo_status_string", "fo_last_error"):
        assert n in names


@pytest.mark.skipif(not (os.path.exists(LIB) and os.path.exists(PROBE_LIB)), reason="library not built")
def test_library_exports_every_declared_symbol():
    headers = [os.path.basename(h) for h in glob.glob(os.path.join(ROOT, "include", "*.h"))]
    for h in headers:
        lib = ctypes.CDLL(LIB_OF_HEADER.get(h, LIB))
        missing = [n for n in declared_functions([h]) if not hasattr(lib, n)]
        assert not missing, (h, missing)
    assert declared_functions(["fo_probe.h"]) == ["fo_probe_copy", "fo_probe_fma64", "fo_probe_read", "fo_probe_write"]


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


def _bad_mesh_cases():
    """(name, mesh, expected status, message fragment) for descriptors fo_mesh_create rejects
    during host-side validation, before any device call."""
    from dataclasses import replace

    import numpy as np

    from fo_inputs import structured_box
    from fo_inputs.meshgen import ExtrudedMesh

    xy, cells, sigma = structured_box(3, 2, 2, 3e3, 2e3, elem="wedge")
    V = xy.shape[0]
    good = ExtrudedMesh("wedge", xy, cells, np.full(V, 1000.0), np.full(V, 800.0), np.full(V, 500.0), sigma)
    H0 = good.thickness.copy(); H0[3] = 0.0
    bneg = good.beta.copy(); bneg[1] = -1.0
    cw = good.cells.copy(); cw[0] = cw[0][::-1]
    oob = good.cells.copy(); oob[2, 1] = V + 5
    rep = good.cells.copy(); rep[1, 2] = rep[1, 0]
    # a fan of 70 triangles around one vertex: more than 64 cells at a vertex
    ang = np.linspace(0, 2 * np.pi, 71)[:-1]
    fxy = np.vstack([[0.0, 0.0], np.stack([1e3 * np.cos(ang), 1e3 * np.sin(ang)], 1)])
    fcells = np.array([[0, 1 + i, 1 + (i + 1) % 70] for i in range(70)], dtype=np.int32)
    nf = fxy.shape[0]
    fan = ExtrudedMesh("wedge", fxy, fcells, np.full(nf, 1000.0), np.full(nf, 800.0), np.full(nf, 500.0),
                       np.linspace(0, 1, 3))
    # an extra vertex that no cell uses
    lone = replace(good, xy=np.vstack([good.xy, [[9e3, 9e3]]]), surface=np.append(good.surface, 1000.0),
                   thickness=np.append(good.thickness, 800.0), beta=np.append(good.beta, 500.0))
    return [
        ("zero thickness", replace(good, thickness=H0), -4, b"thickness"),
        ("vertex in no cell", lone, -4, b"no base cell"),
        ("negative beta", replace(good, beta=bneg), -4, b"beta"),
        ("clockwise cell", replace(good, cells=cw), -4, b"counter-clockwise"),
        ("vertex id out of range", replace(good, cells=oob), -1, b"out of range"),
        ("repeated vertex", replace(good, cells=rep), -4, b"repeated vertex"),
        ("sigma not increasing", replace(good, sigma=np.array([0.0, 0.6, 0.4, 1.0])), -4, b"sigma"),
        ("sigma not ending at 1", replace(good, sigma=np.array([0.0, 0.5, 0.9])), -4, b"sigma"),
        ("no layers", replace(good, sigma=np.array([0.0])), -1, b"L >= 1"),
        ("non-positive A", replace(good, A=0.0), -1, b"constants"),
        ("Glen exponent below 1", replace(good, n=0.5), -1, b"constants"),
        ("more than 64 cells at a vertex", fan, -1, b"more than 64"),
    ]


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("case", _bad_mesh_cases(), ids=lambda c: c[0])
def test_mesh_validation_rejects_without_gpu(case):
    from paper_2204_04321_amd import _lib
    from paper_2204_04321_amd.api import mesh_desc
    name, m, status, frag = case
    keep = []
    d = mesh_desc(m, keep)
    out = ctypes.c_void_p()
    assert _lib.lib().fo_mesh_create(ctypes.byref(d), None, ctypes.byref(out)) == status, name
    assert frag in _lib.lib().fo_last_error(), (name, _lib.lib().fo_last_error())
    assert not out.value


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_plain_c_caller(tmp_path):
    """The ABI is usable from C: compile the example against the header, link the library,
    run the host-side calls."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    exe = str(tmp_path / "abi_check")
    src = os.path.join(ROOT, "paper_2204_04321_amd", "examples", "abi_check.c")
    libdir = os.path.dirname(LIB)
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), src, "-o", exe,
                    "-L", libdir, "-lfo_stokes", "-Wl,-rpath," + libdir], check=True, capture_output=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert p.returncode == 0, p.stdout + p.stderr
    assert "degenerate" in p.stdout
    # the binding's option struct has the C layout and defaults (GMRES, the paper's solver)
    from paper_2204_04321_amd import _lib
    o = _lib.NewtonOpts()
    _lib.lib().fo_newton_default_opts(ctypes.byref(o))
    assert o.linear_solver == _lib.FO_LIN_GMRES and o.gmres_restart == 100
    assert f"linear solver 0, opts size {ctypes.sizeof(_lib.NewtonOpts)}" in p.stdout
    assert f"report size {ctypes.sizeof(_lib.NewtonReport)}" in p.stdout
    assert o.learned_fallback == 1 and o.learned_smooth == 0 and not o.mlp_params
