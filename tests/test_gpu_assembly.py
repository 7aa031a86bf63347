"""GPU parity of the HIP assembly path against the FP64 oracle (through the C ABI).

Bar: FP64 residual and Jacobian within 1e-12 of the oracle, row-scaled by the
assembled absolute element contributions (|dR_i| <= 1e-12 sum_e |R_e,i|,
|dJ_ij| <= 1e-12 max_j sum_e |J_e,ij|); FP32 Jacobian values within 1e-5 on
the same scale; integer pattern bit-exact.
"""
import numpy as np
import pytest
import torch

from fo_inputs import (box_hex_single, config0_slab, config1_icesheet, perturbed, right_wedge_single,
                       smooth_velocity, structured_box)
from fo_inputs.meshgen import ExtrudedMesh, _dome_fields, dome_velocity, ellipse_mesh
from oracle import fo_oracle as fo
from oracle import solve

from gpu_util import gpu_jacobian, gpu_mesh, gpu_residual, row_scaled_errors, to_dev

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


def _small_ellipse(seed=5, n_points=300, L=7):
    rng = np.random.default_rng(seed)
    a, b = 60e3, 35e3
    xy, tri = ellipse_mesh(n_points, a, b, rng)
    s, H, beta = _dome_fields(xy, a, b, rng, 2500.0, 400.0, 500.0, 1.0, 15e3, 60e3)
    m = ExtrudedMesh("wedge", xy, tri, s, H, beta, np.linspace(0, 1, L + 1), A=1.3e-16)
    return m, dome_velocity(m, a, b, rng, 200.0)


def _box(nx, ny, L, elem, seed):
    xy, cells, sigma = structured_box(nx, ny, L, 5e3, 4e3, elem=elem)
    x, y = xy[:, 0], xy[:, 1]
    H = 700 + 150 * np.sin(x / 2e3) * np.cos(y / 1.5e3)
    m = ExtrudedMesh(elem, xy, cells, 300 - 0.02 * x + H, H, 800 + 0 * x, sigma)
    m = perturbed(m, np.random.default_rng(seed), 0.2)
    return m, smooth_velocity(m, np.random.default_rng(seed), 80.0, 0.05)


def _graded_sigma(m):
    L = m.n_layers
    sg = 1 - (1 - np.linspace(0, 1, L + 1)) ** 1.5    # thinner layers at the bed
    sg[0], sg[-1] = 0.0, 1.0
    return m.with_fields(sigma=sg)


def _fan(n_cells=64, L=3, seed=8):
    """One vertex in n_cells triangles (64 is the per-vertex maximum), ring vertices with 2 or 3 cells."""
    rng = np.random.default_rng(seed)
    ang = np.sort(rng.uniform(0, 2 * np.pi, n_cells))
    r = 3e3 * (1 + 0.2 * rng.uniform(-1, 1, n_cells))
    xy = np.vstack([[0.0, 0.0], np.stack([r * np.cos(ang), r * np.sin(ang)], 1)])
    cells = np.array([[0, 1 + i, 1 + (i + 1) % n_cells] for i in range(n_cells)], dtype=np.int32)
    V = xy.shape[0]
    H = 600 + 100 * rng.uniform(size=V)
    m = ExtrudedMesh("wedge", xy, cells, 200 - 0.01 * xy[:, 0] + H, H, 400 + 300 * rng.uniform(size=V),
                     np.linspace(0, 1, L + 1))
    return m, smooth_velocity(m, rng, 60.0, 0.05)


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


@pytest.mark.parametrize("kind", ["newton", "picard"])
def test_jacobian_f64_parity(case, kind):
    name, m, U, M = case
    R, J = gpu_jacobian(M, U, "f64", kind)
    Ro, Jo = fo.assemble(m, U, picard=(kind == "picard"))
    rs, js = fo.abs_scales(m, U, picard=(kind == "picard"))
    er, ej = row_scaled_errors(R, J, Ro, Jo, rs, js)
    print(f"[{name}/{kind}] row-scaled err R {er:.2e} J {ej:.2e}; "
          f"plain |dJ|/|J| {abs(J - Jo).max() / abs(Jo).max():.2e}")
    assert er <= TOL64 and ej <= TOL64


def test_residual_f64_parity(case):
    name, m, U, M = case
    R = gpu_residual(M, U)
    Ro = fo.residual(m, U)
    rs, _ = fo.abs_scales(m, U)
    er = np.max(np.abs(R - Ro) / rs)
    assert er <= TOL64


def test_jacobian_f32_bound(case):
    name, m, U, M = case
    R, J = gpu_jacobian(M, U, "f32", "newton")
    Ro, Jo = fo.assemble(m, U)
    rs, js = fo.abs_scales(m, U)
    er, ej = row_scaled_errors(R, J, Ro, Jo, rs, js)
    print(f"[{name}/f32] residual (FP64) err {er:.2e}, FP32 J row-scaled err {ej:.2e}")
    assert er <= TOL64      # residual stays FP64
    assert ej <= TOL32


def test_sia_parity(case):
    name, m, U, M = case
    Ug = M.sia()
    torch.cuda.synchronize()
    Uo = solve.sia_guess(m)
    scale = np.abs(Uo).max() + 1e-300
    assert np.abs(Ug.cpu().numpy() - Uo).max() <= 1e-12 * scale


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


def test_icesheet_full_size_sampled_rows():
    """Ice-sheet configuration (~2.5M wedges) in the benchmark's launch configuration:
    sampled Jacobian rows and residual entries against the oracle on the cells around
    them, plus symmetry J_ij = J_ji on sampled entries."""
    m, U = config1_icesheet()
    print(f"\n[case] icesheet: cells={m.n_cells} dofs={m.n_dofs}", flush=True)
    M = gpu_mesh(m)
    Ud = to_dev(U)
    R, Jv = M.jacobian(Ud)
    rowptr, colidx = M.pattern()
    torch.cuda.synchronize()
    R = R.cpu().numpy()
    Jv = Jv.cpu().numpy()
    rowptr = rowptr.cpu().numpy()
    colidx = colidx.cpu().numpy()
    rng = np.random.default_rng(123)
    L = m.n_layers
    sel = np.unique(np.concatenate([
        rng.choice(m.n_dofs, 48, replace=False),
        [0, 1, m.n_dofs - 1, m.n_dofs - 2],
        2 * (rng.choice(m.n_verts, 6) * (L + 1)),          # bed rows
        2 * (rng.choice(m.n_verts, 6) * (L + 1) + L) + 1,  # surface rows
    ]))
    r_o, J_o, cells = fo.assemble_rows(m, U, sel)
    rs, js = fo.abs_scales(m, U, cells=cells)
    for n, i in enumerate(sel):
        cols = colidx[rowptr[i]:rowptr[i + 1]]
        vals = Jv[rowptr[i]:rowptr[i + 1]]
        ref = J_o[n].toarray().ravel()
        assert np.array_equal(np.sort(J_o[n].indices), cols)
        assert np.max(np.abs(vals - ref[cols])) <= TOL64 * js[i], i
        assert abs(R[i] - r_o[n]) <= TOL64 * rs[i], i
    # symmetry on sampled entries (the Jacobian is the Hessian of an energy)
    for i in rng.choice(m.n_dofs, 200, replace=False):
        cols = colidx[rowptr[i]:rowptr[i + 1]]
        for jj in cols[:: max(1, len(cols) // 6)]:
            p = rowptr[i] + np.searchsorted(cols, jj)
            cj = colidx[rowptr[jj]:rowptr[jj + 1]]
            q = rowptr[jj] + np.searchsorted(cj, i)
            assert colidx[q] == i
            assert abs(Jv[p] - Jv[q]) <= 1e-12 * max(abs(Jv[p]), abs(Jv[rowptr[i]:rowptr[i + 1]]).max())
    # the FP32 Jacobian in the same launch configuration, on the same sampled rows
    R32, J32 = M.jacobian(Ud, dtype="f32")
    torch.cuda.synchronize()
    R32 = R32.cpu().numpy()
    J32 = J32.cpu().numpy().astype(np.float64)
    for n, i in enumerate(sel):
        cols = colidx[rowptr[i]:rowptr[i + 1]]
        ref = J_o[n].toarray().ravel()
        assert np.max(np.abs(J32[rowptr[i]:rowptr[i + 1]] - ref[cols])) <= TOL32 * js[i], i
        assert abs(R32[i] - r_o[n]) <= TOL64 * rs[i], i
