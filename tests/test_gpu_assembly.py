"""GPU parity of the HIP assembly path against the FP64 oracle (through the C ABI).

Bars, each asserted (FP64):
  * row-scaled by the per-term scale S (the sum of the absolute values of every
    quadrature-point term summed into the entry; it bounds the rounding error of any
    summation order): |dR_i| <= 1e-12 S^R_i, |dJ_ij| <= 1e-12 max_j S^J_ij;
  * row-scaled by the element-level scale: |dR_i| <= TOL64_ELEM sum_e |R_e,i|,
    |dJ_ij| <= TOL64_ELEM max_j sum_e |J_e,ij| (looser than S where the terms of one
    element cancel);
  * norm-wise: ||dR||_inf <= 1e-12 ||R||_inf, max |dJ| <= 1e-12 max |J|.
FP32 Jacobian values: 1e-5 on the per-term and element-level scales, 1e-6 norm-wise.
Integer pattern bit-exact.
"""
import numpy as np
import pytest
import torch

from fo_inputs import (box_hex_single, config0_slab, config1_icesheet, floating_slab, marine_sheet, perturbed,
                       right_wedge_single, smooth_velocity, structured_box)
from fo_inputs.meshgen import ExtrudedMesh, _dome_fields, dome_velocity, ellipse_mesh
from oracle import fo_oracle as fo
from oracle import solve

from gpu_util import gpu_jacobian, gpu_mesh, gpu_residual, parity_errors, to_dev

pytestmark = pytest.mark.gpu

TOL64 = 1e-12        # per-term row scale and norm-wise
TOL64_ELEM = 1e-12   # element-level row scale
TOL32 = 1e-5         # FP32 Jacobian, row scales
TOL32_PLAIN = 1e-6   # FP32 Jacobian, norm-wise


def _small_ellipse(seed=5, n_points=300, L=7, elem="wedge"):
    rng = np.random.default_rng(seed)
    a, b = 60e3, 35e3
    xy, tri = ellipse_mesh(n_points, a, b, rng)
    s, H, beta = _dome_fields(xy, a, b, rng, 2500.0, 400.0, 500.0, 1.0, 15e3, 60e3)
    m = ExtrudedMesh(elem, xy, tri, s, H, beta, np.linspace(0, 1, L + 1), A=1.3e-16)
    return m, dome_velocity(m, a, b, rng, 200.0)


def _box(nx, ny, L, elem, seed):
    xy, cells, sigma = structured_box(nx, ny, L, 5e3, 4e3, elem=elem)
    x, y = xy[:, 0], xy[:, 1]
    H = 700 + 150 * np.sin(x / 2e3) * np.cos(y / 1.5e3)
    m = ExtrudedMesh(elem, xy, cells, 300 - 0.02 * x + H, H, 800 + 0 * x, sigma)
    m = perturbed(m, np.random.default_rng(seed), 0.2)
    return m, smooth_velocity(m, np.random.default_rng(seed), 80.0, 0.05)


def _thin_margin(elem, seed):
    """Thickness falling from 900 m to 1 m across the box (a land-terminating margin): the
    thinnest columns have layers 0.1 m thick under cells 0.6 km wide."""
    xy, cells, sigma = structured_box(8, 4, 10, 5e3, 2e3, elem=elem)
    x = xy[:, 0]
    H = 1.0 + 899.0 * (1.0 - x / 5e3) ** 2
    m = ExtrudedMesh(elem, xy, cells, 200 + H, H, 500 + 0 * x, sigma)
    m = perturbed(m, np.random.default_rng(seed), 0.2)
    return m, smooth_velocity(m, np.random.default_rng(seed), 60.0, 0.05)


def _graded_sigma(m):
    L = m.n_layers
    sg = 1 - (1 - np.linspace(0, 1, L + 1)) ** 1.5    # thinner layers at the bed
    sg[0], sg[-1] = 0.0, 1.0
    return m.with_fields(sigma=sg)


def _fan(n_cells=64, L=3, seed=8, elem="wedge"):
    """One vertex in n_cells triangles (64 is the per-vertex maximum), ring vertices with 2 or 3 cells."""
    rng = np.random.default_rng(seed)
    ang = np.sort(rng.uniform(0, 2 * np.pi, n_cells))
    r = 3e3 * (1 + 0.2 * rng.uniform(-1, 1, n_cells))
    xy = np.vstack([[0.0, 0.0], np.stack([r * np.cos(ang), r * np.sin(ang)], 1)])
    cells = np.array([[0, 1 + i, 1 + (i + 1) % n_cells] for i in range(n_cells)], dtype=np.int32)
    V = xy.shape[0]
    H = 600 + 100 * rng.uniform(size=V)
    m = ExtrudedMesh(elem, xy, cells, 200 - 0.01 * xy[:, 0] + H, H, 400 + 300 * rng.uniform(size=V),
                     np.linspace(0, 1, L + 1))
    return m, smooth_velocity(m, rng, 60.0, 0.05)


def _float_slab(elem, steep=False, seed=14):
    """Floating slab, every side an ocean front; steep: thickness alternating 40 m / 2000 m
    between neighbouring vertices (layers of a front face differ 50x in thickness)."""
    m = floating_slab(elem, nx=5, ny=4, n_layers=4, jitter=0.2, seed=seed)
    if steep:
        H = np.where((np.round(m.xy[:, 0] / 6e3) + np.round(m.xy[:, 1] / 5e3)) % 2 == 0, 40.0, 2000.0)
        m = m.with_fields(thickness=H, surface=(1 - m.rho / m.rho_w) * H)
    return m, smooth_velocity(m, np.random.default_rng(seed), 150.0, 0.05)


def _free_slip_patch(seed=9):
    """beta = 0 on part of the bed (free slip there)."""
    m, U = _box(5, 4, 3, "wedge", seed)
    beta = m.beta.copy()
    beta[m.xy[:, 0] < 2e3] = 0.0
    return m.with_fields(beta=beta), U


CASES = {
    "slab_hex_2000": lambda: config0_slab(),
    "ellipse_wedge_ragged": lambda: _small_ellipse(),
    "box_wedge_pert": lambda: _box(5, 4, 3, "wedge", 1),
    "box_hex_pert": lambda: _box(3, 3, 2, "hex", 2),
    "single_layer_wedge": lambda: _box(4, 3, 1, "wedge", 3),
    "single_layer_hex": lambda: _box(3, 2, 1, "hex", 4),
    "graded_sigma_wedge": lambda: (lambda mu: (_graded_sigma(mu[0]), mu[1]))(_box(4, 4, 5, "wedge", 5)),
    "one_hex": lambda: (box_hex_single(700., 400., 300., 250.),
                        np.random.default_rng(6).normal(size=16) * 30),
    "one_wedge": lambda: (right_wedge_single(600., 900., 250., 300.),
                          np.random.default_rng(7).normal(size=12) * 30),
    # Glen exponents other than 3 take the general power-law viscosity path
    "glen_n1_wedge": lambda: (lambda mu: (mu[0].with_fields(n=1.0, A=2e-13), mu[1]))(_box(4, 3, 3, "wedge", 10)),
    "glen_n4_wedge": lambda: (lambda mu: (mu[0].with_fields(n=4.0, A=1e-20), mu[1]))(_box(5, 4, 4, "wedge", 13)),
    "glen_n2p5_hex": lambda: (lambda mu: (mu[0].with_fields(n=2.5, A=3e-15), mu[1]))(_box(3, 3, 2, "hex", 11)),
    "fan_64_cells_at_a_vertex": lambda: _fan(),
    "ellipse_wedge_20_layers": lambda: _small_ellipse(seed=12, n_points=200, L=20),
    "free_slip_patch": lambda: _free_slip_patch(),
    # tetrahedral extrusion: 3 tetrahedra per prism, split by the global vertex order
    "tet_box_pert": lambda: _box(5, 4, 3, "tet", 15),
    "tet_ellipse_ragged": lambda: _small_ellipse(seed=16, n_points=250, L=6, elem="tet"),
    "tet_single_layer": lambda: _box(4, 3, 1, "tet", 17),
    "tet_graded_sigma": lambda: (lambda mu: (_graded_sigma(mu[0]), mu[1]))(_box(3, 4, 5, "tet", 18)),
    "tet_fan_64_cells": lambda: _fan(elem="tet"),
    "tet_glen_n1": lambda: (lambda mu: (mu[0].with_fields(n=1.0, A=2e-13), mu[1]))(_box(4, 3, 3, "tet", 19)),
    "tet_glen_n4": lambda: (lambda mu: (mu[0].with_fields(n=4.0, A=1e-20), mu[1]))(_box(4, 4, 3, "tet", 20)),
    # degenerate velocity: U = 0 gives exactly zero strain rates, so the viscosity sits at its
    # regularised cap and the Newton term of the Jacobian vanishes (a rigid translation is
    # pinned on the oracle only: its strain rates are rounding noise that the cap amplifies)
    "zero_velocity_wedge": lambda: (lambda mu: (mu[0], np.zeros_like(mu[1])))(_box(4, 3, 3, "wedge", 21)),
    "thin_margin_wedge": lambda: _thin_margin("wedge", 23),
    "thin_margin_tet": lambda: _thin_margin("tet", 24),
    # ocean back-pressure on marked lateral fronts; floating ice has beta = 0
    "ocean_front_slab_hex": lambda: _float_slab("hex"),
    "ocean_front_slab_wedge_steep": lambda: _float_slab("wedge", steep=True),
    "ocean_front_marine_sheet": lambda: marine_sheet(seed=3, n_points=500, n_layers=5),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    m, U = CASES[request.param]()
    print(f"\n[case] {request.param}: elem={m.elem} cells={m.n_cells} dofs={m.n_dofs}", flush=True)
    M = gpu_mesh(m)
    return request.param, m, U, M


def test_pattern_matches_oracle(case):
    name, m, U, M = case
    rowptr, colidx = M.pattern()
    rp, ci = fo.jacobian_pattern(m)
    assert M.nnz == ci.shape[0]
    np.testing.assert_array_equal(rowptr.cpu().numpy(), rp)
    np.testing.assert_array_equal(colidx.cpu().numpy().astype(np.int64), ci)


def _report(tag, e):
    print(f"[{tag}] R: term {e['term'][0]:.2e} elem {e['elem'][0]:.2e} plain {e['plain'][0]:.2e} | "
          f"J: term {e['term'][1]:.2e} elem {e['elem'][1]:.2e} plain {e['plain'][1]:.2e} | "
          f"worst elem rows R {e['worst_elem'][0]} J {e['worst_elem'][1]}")


@pytest.mark.parametrize("kind", ["newton", "picard"])
def test_jacobian_f64_parity(case, kind):
    name, m, U, M = case
    pic = kind == "picard"
    R, J = gpu_jacobian(M, U, "f64", kind)
    Ro, Jo = fo.assemble(m, U, picard=pic)
    e = parity_errors(R, J, Ro, Jo, fo.abs_scales(m, U, picard=pic), fo.element_scales(m, U, picard=pic))
    _report(f"{name}/{kind}", e)
    assert max(e["term"]) <= TOL64
    assert max(e["elem"]) <= TOL64_ELEM
    assert max(e["plain"]) <= TOL64


def test_residual_f64_parity(case):
    name, m, U, M = case
    R = gpu_residual(M, U)
    Ro = fo.residual(m, U)
    rs, _ = fo.abs_scales(m, U)
    er_, _ = fo.element_scales(m, U)
    d = np.abs(R - Ro)
    term, elem, plain = (d / rs).max(), (d / er_).max(), d.max() / np.abs(Ro).max()
    print(f"[{name}/residual] term {term:.2e} elem {elem:.2e} plain {plain:.2e}")
    assert term <= TOL64 and elem <= TOL64_ELEM and plain <= TOL64


def test_jacobian_f32_bound(case):
    name, m, U, M = case
    R, J = gpu_jacobian(M, U, "f32", "newton")
    Ro, Jo = fo.assemble(m, U)
    e = parity_errors(R, J, Ro, Jo, fo.abs_scales(m, U), fo.element_scales(m, U))
    _report(f"{name}/f32", e)
    # the residual stays FP64
    assert e["term"][0] <= TOL64 and e["elem"][0] <= TOL64_ELEM and e["plain"][0] <= TOL64
    assert e["term"][1] <= TOL32 and e["elem"][1] <= TOL32 and e["plain"][1] <= TOL32_PLAIN


def test_sia_parity(case):
    """Shallow-ice guess against the oracle's.  Where beta = 0 the sliding speed is the cap
    in the direction of -grad s, which is undefined where grad s vanishes (a flat floating
    slab): those columns, where either side's gradient is rounding noise, are left out."""
    name, m, U, M = case
    Ug = M.sia()
    torch.cuda.synchronize()
    Uo = solve.sia_guess(m)
    gx, gy = solve.vertex_surface_gradient(m)
    ill = (m.beta == 0) & (np.hypot(gx, gy) <= 1e-12)
    keep = ~np.repeat(ill, 2 * (m.n_layers + 1))
    scale = np.abs(Uo).max() + 1e-300
    d = np.abs(Ug.cpu().numpy() - Uo)[keep]
    assert d.size == 0 or d.max() <= 1e-12 * scale


def test_repeatability(case):
    """Owner-computes assembly has no global atomics: two runs are bitwise identical."""
    name, m, U, M = case
    R1, J1 = gpu_jacobian(M, U)
    R2, J2 = gpu_jacobian(M, U)
    assert np.array_equal(J1.data, J2.data)
    assert np.array_equal(R1, R2)
    assert np.array_equal(gpu_residual(M, U), R1)


def test_outputs_fully_overwritten(case):
    """No zero fill is needed: stale values in the output buffers never leak through."""
    name, m, U, M = case
    Ud = to_dev(U)
    R0, J0 = M.jacobian(Ud)
    Rn = torch.full_like(R0, float("nan"))
    Jn = torch.full_like(J0, float("nan"))
    M.jacobian(Ud, R=Rn, Jvals=Jn)
    torch.cuda.synchronize()
    assert torch.equal(Rn, R0) and torch.equal(Jn, J0)


def _full_mesh_parity(factory, label, elem_tol=TOL64_ELEM):
    """Every residual entry and every Jacobian value, FP64 and FP32, of the mesh `factory`
    builds, in the benchmark's launch configuration, against the oracle.  The oracle rows of
    each range of vertex columns come from the cells around them, in host processes started
    by "spawn" (they never touch the device) that read the GPU arrays from files."""
    import multiprocessing as mp
    import os
    import shutil
    import time

    import oracle_pool
    m, U = factory()
    print(f"\n[case] {label}: cells={m.n_cells} elem={m.elem} dofs={m.n_dofs}", flush=True)
    M = gpu_mesh(m)
    Ud = to_dev(U)
    R, Jv = M.jacobian(Ud)
    R32, J32 = M.jacobian(Ud, dtype="f32")
    rowptr, colidx = M.pattern()
    torch.cuda.synchronize()
    d = oracle_pool.scratch_dir()
    try:
        files = {}
        for k, t in (("R", R), ("J", Jv), ("J32", J32), ("rowptr", rowptr), ("colidx", colidx)):
            files[k] = os.path.join(d, k + ".npy")
            np.save(files[k], t.cpu().numpy())
        # the FP32 pass writes the same FP64 residual
        assert torch.equal(R, R32)
        del Jv, J32
        t0 = time.perf_counter()
        workers = min(16, len(os.sched_getaffinity(0)))
        with mp.get_context("spawn").Pool(workers, initializer=oracle_pool.init_worker,
                                          initargs=(factory, files)) as pool:
            res = pool.map(oracle_pool.compare_columns, oracle_pool.column_ranges(m.n_verts, 8 * workers),
                           chunksize=1)
        tot = oracle_pool.merge(res)
        print(f"[{label}] oracle comparison of {tot['rows']} rows on {workers} processes in "
              f"{time.perf_counter() - t0:.1f} s", flush=True)
    finally:
        shutil.rmtree(d, ignore_errors=True)
    for key in ("R", "J", "J32"):
        t = tot[key]
        print(f"[{label}/{key}] term {t['term']:.2e} (row {t['term_row']}), elem {t['elem']:.2e} "
              f"(row {t['elem_row']}), plain {t['plain']:.2e}", flush=True)
    assert tot["pattern_ok"] and tot["rows"] == m.n_dofs
    for key in ("R", "J"):
        t = tot[key]
        assert t["term"] <= TOL64 and t["elem"] <= elem_tol and t["plain"] <= TOL64, (key, t)
    t = tot["J32"]
    assert t["term"] <= TOL32 and t["elem"] <= TOL32 and t["plain"] <= TOL32_PLAIN, t


def test_icesheet_full_mesh_parity():
    """Ice-sheet configuration (2,487,040 wedges, 2,750,000 dofs, 108M nonzeros), whole mesh."""
    _full_mesh_parity(config1_icesheet, "icesheet")


def test_icesheet_tetrahedra_full_mesh_parity():
    """The same mesh extruded to tetrahedra (7,461,120 of them), as `bench.py --workload tet`
    assembles it, whole mesh."""
    import oracle_pool
    _full_mesh_parity(oracle_pool.icesheet_tetrahedra, "icesheet_tet")


def test_sia_guess_full_size():
    """The shallow-ice guess of every column of the ice-sheet mesh and of the benchmarked
    marine sheet (floating shelf included) against the oracle's (columns with beta = 0 and a
    vanishing surface gradient left out, as in test_sia_parity)."""
    import oracle_pool
    for factory in (config1_icesheet, oracle_pool.marine_bench_sheet):
        m, _ = factory()
        M = gpu_mesh(m)
        Ug = M.sia().cpu().numpy()
        Uo = solve.sia_guess(m)
        gx, gy = solve.vertex_surface_gradient(m)
        keep = ~np.repeat((m.beta == 0) & (np.hypot(gx, gy) <= 1e-12), 2 * (m.n_layers + 1))
        err = np.abs(Ug - Uo)[keep].max() / np.abs(Uo).max()
        print(f"\n[sia full size] {m.name or factory.__name__}: {m.n_dofs} dofs, {err:.1e}", flush=True)
        assert keep.sum() > 0.9 * keep.size and err <= 1e-12
        M.close()


def test_marine_sheet_full_mesh_parity():
    """The marine ice sheet of `bench.py --workload marine` (125k base points, 10 layers, a
    floating shelf with beta = 0 and ocean fronts on its seaward margin), whole mesh.  The
    per-term and norm-wise bars are 1e-12; the element-level bar is 2e-12 on this mesh.  Its
    worst row (residual row 1244541: a front vertex of the floating shelf, H = 60 m, in plug
    flow at about 1e4 m/yr whose velocity changes by 0.6 m/yr between levels 6 m apart) takes
    its vertical shear from velocities that agree to 1e-4, so both sides carry about 1e-12
    relative rounding in it before any sum; there the per-term scale is 5.2 times the
    element-level one, and the row lies at 1.6e-12 of the element-level scale and 3e-13 of the
    per-term scale."""
    import oracle_pool
    _full_mesh_parity(oracle_pool.marine_bench_sheet, "marine", elem_tol=2e-12)


def _cell_of(m, U, t, k):
    """Base cell t at layer k of an extruded mesh as a one-cell, one-layer mesh with the same
    corner coordinates, elevations and velocities (bed friction only for k = 0)."""
    vs = m.cells[t]
    b = m.surface[vs] - m.thickness[vs]
    z0 = b + m.sigma[k] * m.thickness[vs]
    z1 = b + m.sigma[k + 1] * m.thickness[vs]
    beta = m.beta[vs] if k == 0 else np.zeros(len(vs))
    one = ExtrudedMesh(m.elem, m.xy[vs], np.arange(len(vs), dtype=np.int32)[None, :], z1, z1 - z0, beta,
                       np.array([0.0, 1.0]), A=m.A, n=m.n)
    L1 = m.n_layers + 1
    Uc = U.reshape(-1, 2)[(vs[:, None] * L1 + np.array([k, k + 1])[None, :]).ravel()]
    # reorder to the one-cell mesh's node numbering: vertex i, level 0 or 1 -> node 2 i + lev
    return one, Uc.reshape(-1)


def test_fp32_element_matrix_error_on_icesheet_cells():
    """The FP32-Jacobian variant's error per element matrix, max |dJ_e| / max |J_e|, on 256
    seeded cells of the ice-sheet configuration (each assembled alone, so the assembled
    matrix is the element matrix), against the FP64 oracle."""
    m, U = config1_icesheet()
    rng = np.random.default_rng(77)
    worst, errs = 0.0, []
    for t, k in zip(rng.choice(m.n_base_cells, 256, replace=False), rng.integers(0, m.n_layers, 256)):
        one, Uc = _cell_of(m, U, t, int(k))
        M = gpu_mesh(one)
        _, J32 = gpu_jacobian(M, Uc, "f32")
        _, Jo = fo.assemble(one, Uc)
        e = abs(J32 - Jo).max() / abs(Jo).max()
        errs.append(e)
        M.close()
    errs = np.array(errs)
    print(f"\n[icesheet cells, FP32 element matrices] max rel error {errs.max():.2e}, median {np.median(errs):.2e}")
    assert errs.max() <= 1e-5


def test_single_mesh_beyond_int32_offsets():
    """One mesh whose Jacobian has more than 2^31 entries (a 1649 x 1649 structured wedge grid,
    10 layers: 54.4M wedges, 59.9M dofs, 2.36e9 nonzeros), so every 64-bit offset path of the
    assembly is exercised: residual and Jacobian rows (FP64 and FP32 values) of vertex columns
    at the start, around the row where the offsets pass 2^31, and at the end against the
    oracle's rows from the cells around them (pattern bit for bit, the FP64 and FP32 bars of
    this file on those rows); then a Newton solve of the whole mesh (GMRES with the two-level
    preconditioner, whose setup and application, like the SpMV, read J and J P0 through
    64-bit offsets) must converge."""
    from paper_2204_04321_amd.api import Mdsc
    nx = 1649
    L = 10
    xy, cells, sigma = structured_box(nx, nx, L, 4000e3, 4000e3, elem="wedge")
    x, y = xy[:, 0], xy[:, 1]
    H = 1500 + 500 * np.sin(x / 2e5) * np.cos(y / 1.5e5)
    m = ExtrudedMesh("wedge", xy, cells, 300 - 2e-4 * x + H, H, 800 + 0 * x, sigma)
    U = smooth_velocity(m, np.random.default_rng(3), 80.0, 0.05)
    print(f"\n[case] int64 offsets: cells={m.n_cells} dofs={m.n_dofs}", flush=True)
    M = gpu_mesh(m)
    assert M.nnz > 2 ** 31, M.nnz
    Ud = to_dev(U)
    R, Jv = M.jacobian(Ud)
    R32, J32 = M.jacobian(Ud, dtype="f32")
    rowptr, colidx = M.pattern()
    torch.cuda.synchronize()
    assert torch.equal(R, R32)
    nb = 2 * (L + 1)
    cross = int(torch.searchsorted(rowptr, torch.tensor([2 ** 31], device=rowptr.device)).item()) - 1
    vc = cross // nb
    V = m.n_verts
    verts = np.unique(np.array([0, 1, nx + 2, vc - 1, vc, vc + 1, V - nx - 3, V - 2, V - 1]))
    dofs = (verts[:, None] * nb + np.arange(nb)[None, :]).ravel()
    print(f"[int64 offsets] nnz {M.nnz}, offsets pass 2^31 in row {cross} (vertex {vc}); "
          f"{dofs.size} rows checked", flush=True)
    d_t = torch.from_numpy(dofs).to(rowptr.device)
    lo, hi = rowptr[d_t], rowptr[d_t + 1]
    idx = torch.cat([torch.arange(int(a), int(b), device=rowptr.device) for a, b in zip(lo.tolist(), hi.tolist())])
    assert int(hi.max()) > 2 ** 31 and int(lo.min()) < 2 ** 31
    ptr = np.concatenate([[0], np.cumsum((hi - lo).cpu().numpy())])
    g_cols = colidx[idx].cpu().numpy().astype(np.int64)
    g64 = Jv[idx].cpu().numpy()
    g32 = J32[idx].double().cpu().numpy()
    gR = R[d_t].cpu().numpy()
    del Jv, J32
    Ro, Jo, cs = fo.assemble_rows(m, U, dofs)
    rs, js = fo.abs_scales(m, U, cells=cs)
    er, ej = fo.element_scales(m, U, cells=cs)
    assert np.array_equal(Jo.indptr, ptr) and np.array_equal(Jo.indices, g_cols)
    rows = np.repeat(np.arange(dofs.size), np.diff(ptr))
    dR = np.abs(gR - Ro)
    for tag, vals, tol, tol_plain in (("f64", g64, TOL64, TOL64), ("f32", g32, TOL32, TOL32_PLAIN)):
        dJ = np.zeros(dofs.size)
        np.maximum.at(dJ, rows, np.abs(vals - Jo.data))
        e_term, e_elem = (dJ / js[dofs]).max(), (dJ / ej[dofs]).max()
        e_plain = dJ.max() / np.abs(Jo.data).max()
        print(f"[int64 offsets/J {tag}] term {e_term:.2e} elem {e_elem:.2e} plain {e_plain:.2e}", flush=True)
        assert e_term <= tol and e_elem <= tol and e_plain <= tol_plain
    r_term, r_elem = (dR / rs[dofs]).max(), (dR / er[dofs]).max()
    print(f"[int64 offsets/R] term {r_term:.2e} elem {r_elem:.2e}", flush=True)
    assert r_term <= TOL64 and r_elem <= TOL64_ELEM
    del R, R32, rowptr, colidx, idx
    torch.cuda.empty_cache()
    Un = torch.zeros(M.n_dofs, dtype=torch.float64, device="cuda")
    P = Mdsc(M)
    rep = M.newton_solve(Un, tol=1e-8, init="sia", preconditioner="mdsc", mdsc=P)
    print(f"[int64 offsets/newton] status {rep['status']} its {rep['newton_its']} gmres {rep['lin_its']} "
          f"rel {rep['final_rel']:.1e}, {rep['ms_total_solve']:.0f} ms", flush=True)
    assert rep["status"] == 0 and rep["final_rel"] <= 1e-8
    P.close()
    M.close()
