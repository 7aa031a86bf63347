"""The library's ocean-front loads (host code run at mesh upload, fo_front.cpp) against the
oracle, without a GPU: a small driver compiled with hipcc for the host calls
fo::build_front_loads on the same descriptors and prints the per-node loads."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from fo_inputs import floating_slab, marine_sheet
from oracle import fo_oracle as fo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2204_04321_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <string>
#include <vector>
#include "fo_internal.h"
namespace fo {
static std::string msg;
void set_error(const std::string &m) { msg = m; }
fo_status fail(fo_status s, const std::string &m) { msg = m; return s; }
}
int main(int argc, char **argv) {
  FILE *f = fopen(argv[1], "r");
  int elem, V, T, L, nfe;
  if (fscanf(f, "%d %d %d %d", &elem, &V, &T, &L) != 4) return 3;
  const int nv = elem == FO_WEDGE6 ? 3 : 4;
  std::vector<double> xy(2 * V), s(V), H(V), sig(L + 1);
  std::vector<int32_t> cells(size_t(T) * nv);
  for (auto &x : xy) if (fscanf(f, "%lf", &x) != 1) return 3;
  for (auto &x : cells) if (fscanf(f, "%d", &x) != 1) return 3;
  for (auto &x : s) if (fscanf(f, "%lf", &x) != 1) return 3;
  for (auto &x : H) if (fscanf(f, "%lf", &x) != 1) return 3;
  for (auto &x : sig) if (fscanf(f, "%lf", &x) != 1) return 3;
  double rho, g, rw;
  if (fscanf(f, "%lf %lf %lf %d", &rho, &g, &rw, &nfe) != 4) return 3;
  std::vector<int32_t> fe(2 * size_t(nfe));
  for (auto &x : fe) if (fscanf(f, "%d", &x) != 1) return 3;
  fo_mesh_desc d{};
  d.elem = elem; d.n_base_verts = V; d.n_base_cells = T; d.n_layers = L;
  d.base_xy = xy.data(); d.base_cells = cells.data(); d.surface = s.data(); d.thickness = H.data();
  d.rho = rho; d.g = g; d.rho_w = rw; d.front_edges = fe.data(); d.n_front_edges = nfe;
  std::vector<int32_t> vtx;
  std::vector<double> load;
  const fo_status st = fo::build_front_loads(&d, sig, vtx, load);
  if (st != FO_OK) { printf("error %d %s\n", int(st), fo::msg.c_str()); return 0; }
  for (size_t i = 0; i < vtx.size(); ++i)
    for (int k = 0; k <= L; ++k)
      printf("%d %d %.17g %.17g\n", vtx[i], k, load[(i * (L + 1) + k) * 2], load[(i * (L + 1) + k) * 2 + 1]);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    d = tmp_path_factory.mktemp("front")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    r = subprocess.run([hipcc, "-O2", "-std=c++17", f"-I{CSRC}", f"-I{os.path.join(ROOT, 'include')}",
                        str(src), os.path.join(CSRC, "fo_front.cpp"), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return str(exe)


def _run(driver, m, tmp_path):
    inp = tmp_path / "desc.txt"
    fe = np.asarray(m.front_edges).reshape(-1, 2)
    with open(inp, "w") as f:
        f.write(f"{6 if m.elem == 'wedge' else 8} {m.n_verts} {m.n_base_cells} {m.n_layers}\n")
        for arr in (m.xy.ravel(), m.cells.ravel(), m.surface, m.thickness, m.sigma):
            f.write(" ".join(repr(float(x)) if arr.dtype.kind == "f" else str(int(x)) for x in arr) + "\n")
        f.write(f"{m.rho!r} {m.g!r} {m.rho_w!r} {fe.shape[0]}\n" + " ".join(str(int(x)) for x in fe.ravel()) + "\n")
    out = subprocess.run([driver, str(inp)], capture_output=True, text=True, check=True).stdout
    if out.startswith("error"):
        return out
    L1 = m.n_layers + 1
    got = np.zeros((m.n_verts, L1, 2))
    for line in out.splitlines():
        v, k, a, b = line.split()
        got[int(v), int(k)] = (float(a), float(b))
    return got.reshape(-1)


def _steep():
    m = floating_slab("hex", nx=5, ny=4, n_layers=4)
    H = np.where((np.round(m.xy[:, 0] / 6e3) + np.round(m.xy[:, 1] / 5e3)) % 2 == 0, 40.0, 2000.0)
    return m.with_fields(thickness=H, surface=(1 - m.rho / m.rho_w) * H)


@pytest.mark.parametrize("which", ["slab_hex", "slab_wedge", "steep", "marine"])
def test_front_loads_match_oracle(driver, tmp_path, which):
    m = {"slab_hex": lambda: floating_slab("hex"), "slab_wedge": lambda: floating_slab("wedge", jitter=0.25, seed=3),
         "steep": _steep, "marine": lambda: marine_sheet(seed=2, n_points=400, n_layers=4)[0]}[which]()
    got = _run(driver, m, tmp_path)
    ref = fo.front_load(m)
    scale = fo.front_load(m, absolute=True)
    on = scale > 0
    assert np.all(got[~on] == 0.0)
    err = np.abs(got[on] - ref[on]) / scale[on]
    print(f"\n[front loads {which}] max error / per-term scale {err.max():.2e}")
    assert err.max() <= 1e-13


def test_front_edge_validation(driver, tmp_path):
    m = floating_slab("wedge")
    interior = np.array([[m.cells[0, 0], m.cells[0, 2]]], dtype=np.int32)
    assert "shared by two cells" in _run(driver, m.with_fields(front_edges=interior), tmp_path)
    fe = np.asarray(m.front_edges)
    assert "listed twice" in _run(driver, m.with_fields(front_edges=np.vstack([fe, fe[:1, ::-1]])), tmp_path)
    assert "not an edge" in _run(driver, m.with_fields(front_edges=np.array([[0, m.n_verts - 1]])), tmp_path)
