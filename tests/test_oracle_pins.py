"""Pins of the FP64 oracle against facts fixed by the mathematics (no GPU).

Each test targets a mistake that could hide in the oracle: a wrong strain-rate
component or factor (closed-form element matrices, rigid-motion invariance),
a wrong Jacobian term (complex-step and finite differences, symmetry, the
energy whose gradient the residual must be), a wrong viscosity exponent
(homogeneity), wrong gravity or friction signs (closed forms, exact slab
solution in test_oracle_solutions.py).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from fo_inputs import (box_hex_single, config0_slab, perturbed, right_wedge_single,
                       smooth_velocity, structured_box)
from fo_inputs.meshgen import ExtrudedMesh
from oracle import fo_oracle as fo

RG = 910.0 * 9.81


def _box_mesh(nx, ny, L, elem, seed=0, pert=0.25, beta=1000.0, lx=4e3, ly=3e3):
    xy, cells, sigma = structured_box(nx, ny, L, lx, ly, elem=elem)
    rng = np.random.default_rng(seed)
    x, y = xy[:, 0], xy[:, 1]
    H = 800.0 + 100.0 * np.sin(2 * np.pi * x / lx) * np.cos(2 * np.pi * y / ly)
    s = 500.0 - 0.01 * x + 0.004 * y + H
    m = ExtrudedMesh(elem, xy, cells, s, H, np.full(xy.shape[0], beta), sigma)
    if pert:
        m = perturbed(m, rng, pert)
    return m


# --------------------------------------------------------------------------------------
# P-1: closed-form single elements (n = 1: constant viscosity 1/(2A))
# --------------------------------------------------------------------------------------

def _1d(h):
    K = np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    M = np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    C = np.array([[-0.5, -0.5], [0.5, 0.5]])      # C[i, j] = int phi_i' phi_j
    return K, M, C


def test_closed_form_box_hex_n1():
    hx, hy, hz, beta, A = 700.0, 400.0, 300.0, 250.0, 2e-16
    m = box_hex_single(hx, hy, hz, beta=beta)
    m = m.with_fields(n=1.0, A=A)
    sx, sy = -0.02, 0.005
    s_drive = 5.0 + sx * m.xy[:, 0] + sy * m.xy[:, 1]
    U = np.random.default_rng(1).normal(size=m.n_dofs) * 10
    R, J = fo.assemble(m, U, s_drive=s_drive)
    Jd = J.toarray()
    # local node a: vertex i (0:(0,0) 1:(1,0) 2:(1,1) 3:(0,1)) at level k; global node = i*2+k
    ij = {0: (0, 0), 1: (1, 0), 2: (1, 1), 3: (0, 1)}
    Kx, Mx, Cx = _1d(hx)
    Ky, My, Cy = _1d(hy)
    Kz, Mz, Cz = _1d(hz)
    two_mu = 1.0 / A
    ref = np.zeros((16, 16))
    for ia in range(4):
        for ka in range(2):
            for ib in range(4):
                for kb in range(2):
                    xa, ya = ij[ia]
                    xb, yb = ij[ib]
                    ra, rb = 2 * (ia * 2 + ka), 2 * (ib * 2 + kb)
                    xx, yy, zz = Kx[xa, xb] * My[ya, yb] * Mz[ka, kb], Mx[xa, xb] * Ky[ya, yb] * Mz[ka, kb], \
                        Mx[xa, xb] * My[ya, yb] * Kz[ka, kb]
                    # int dN_a/dx dN_b/dy and int dN_a/dy dN_b/dx
                    xy_ = Cx[xa, xb] * Cy[yb, ya] * Mz[ka, kb]
                    yx_ = Cy[ya, yb] * Cx[xb, xa] * Mz[ka, kb]
                    ref[ra, rb] = two_mu * (2 * xx + 0.5 * yy + 0.5 * zz)
                    ref[ra, rb + 1] = two_mu * (xy_ + 0.5 * yx_)
                    ref[ra + 1, rb] = two_mu * (yx_ + 0.5 * xy_)
                    ref[ra + 1, rb + 1] = two_mu * (0.5 * xx + 2 * yy + 0.5 * zz)
                    if ka == 0 and kb == 0:
                        fr = beta * Mx[xa, xb] * My[ya, yb]
                        ref[ra, rb] += fr
                        ref[ra + 1, rb + 1] += fr
    np.testing.assert_allclose(Jd, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
    # n = 1: the residual is affine, F(U) = J U + F(0), F(0) = rho g grad s * V/8 per node
    F0 = fo.residual(m, np.zeros(m.n_dofs), s_drive=s_drive)
    V = hx * hy * hz
    np.testing.assert_allclose(F0[0::2], RG * sx * V / 8, rtol=1e-13)
    np.testing.assert_allclose(F0[1::2], RG * sy * V / 8, rtol=1e-13)
    np.testing.assert_allclose(R, ref @ U + F0, rtol=0, atol=1e-12 * np.abs(R).max())


def test_closed_form_right_wedge_n1():
    hx, hy, hz, beta, A = 600.0, 900.0, 250.0, 300.0, 1e-16
    m = right_wedge_single(hx, hy, hz, beta=beta).with_fields(n=1.0, A=A)
    R, J = fo.assemble(m, np.zeros(m.n_dofs), s_drive=np.zeros(3))
    Jd = J.toarray()
    area = hx * hy / 2
    gl = np.array([[-1 / hx, -1 / hy], [1 / hx, 0.0], [0.0, 1 / hy]])
    MT = area / 12 * np.array([[2.0, 1, 1], [1, 2, 1], [1, 1, 2]])
    Kz, Mz, _ = _1d(hz)
    two_mu = 1.0 / A
    ref = np.zeros((12, 12))
    for ia in range(3):
        for ka in range(2):
            for ib in range(3):
                for kb in range(2):
                    ra, rb = 2 * (ia * 2 + ka), 2 * (ib * 2 + kb)
                    xx = area * gl[ia, 0] * gl[ib, 0] * Mz[ka, kb]
                    yy = area * gl[ia, 1] * gl[ib, 1] * Mz[ka, kb]
                    zz = MT[ia, ib] * Kz[ka, kb]
                    xy_ = area * gl[ia, 0] * gl[ib, 1] * Mz[ka, kb]
                    yx_ = area * gl[ia, 1] * gl[ib, 0] * Mz[ka, kb]
                    ref[ra, rb] = two_mu * (2 * xx + 0.5 * yy + 0.5 * zz)
                    ref[ra, rb + 1] = two_mu * (xy_ + 0.5 * yx_)
                    ref[ra + 1, rb] = two_mu * (yx_ + 0.5 * xy_)
                    ref[ra + 1, rb + 1] = two_mu * (0.5 * xx + 2 * yy + 0.5 * zz)
                    if ka == 0 and kb == 0:
                        ref[ra, rb] += beta * MT[ia, ib]
                        ref[ra + 1, rb + 1] += beta * MT[ia, ib]
    np.testing.assert_allclose(Jd, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


# --------------------------------------------------------------------------------------
# P-2: rigid horizontal motions carry no viscous stress
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("elem", ["hex", "wedge", "tet"])
def test_rigid_motion_invariance(elem):
    m = _box_mesh(3, 3, 3, elem, beta=0.0)
    rng = np.random.default_rng(2)
    U = smooth_velocity(m, rng, 100.0, 0.05)
    xyz = fo.node_xyz(m)
    c1, c2, om = 37.0, -12.0, 3e-3
    rig = np.stack([c1 - om * xyz[:, 1], c2 + om * xyz[:, 0]], axis=1).reshape(-1)
    F1 = fo.residual(m, U)
    F2 = fo.residual(m, U + rig)
    scale = np.abs(F1).max()
    assert np.abs(F2 - F1).max() <= 1e-10 * scale
    # n = 1: constant viscosity, no gravity or friction: exactly zero on the rigid field alone
    m1 = m.with_fields(n=1.0)
    F = fo.residual(m1, rig, s_drive=np.zeros(m.n_verts))
    scale1 = np.abs(fo.residual(m1, U, s_drive=np.zeros(m.n_verts))).max()
    assert np.abs(F).max() <= 1e-11 * scale1
    # and a vertical shear is NOT rigid: it must produce stress
    shear = np.stack([1e-2 * xyz[:, 2], np.zeros(xyz.shape[0])], axis=1).reshape(-1)
    assert np.abs(fo.residual(m1, shear, s_drive=np.zeros(m.n_verts))).max() > 1e-3 * scale1


# --------------------------------------------------------------------------------------
# P-3 / P-4 / P-10 / P-5: symmetry, energy, complex step, finite differences
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("elem", ["hex", "wedge", "tet"])
def test_symmetric_positive_definite(elem):
    m = _box_mesh(2, 2, 3, elem)
    U = smooth_velocity(m, np.random.default_rng(4), 100.0, 0.05)
    for picard in (False, True):
        _, J = fo.assemble(m, U, picard=picard)
        Jd = J.toarray()
        assert np.abs(Jd - Jd.T).max() <= 1e-14 * np.abs(Jd).max()
        np.linalg.cholesky(Jd)      # raises unless SPD


@pytest.mark.parametrize("elem", ["hex", "wedge", "tet"])
def test_residual_is_energy_gradient(elem):
    m = _box_mesh(3, 2, 3, elem)
    rng = np.random.default_rng(5)
    U = smooth_velocity(m, rng, 100.0, 0.05)
    for _ in range(3):
        v = rng.normal(size=U.shape)
        h = 1e-2
        dE = (fo.energy(m, U + h * v) - fo.energy(m, U - h * v)) / (2 * h)
        # fourth-order difference for a tighter check
        dE4 = (8 * (fo.energy(m, U + h * v) - fo.energy(m, U - h * v))
               - (fo.energy(m, U + 2 * h * v) - fo.energy(m, U - 2 * h * v))) / (12 * h)
        Fv = fo.residual(m, U) @ v
        assert abs(dE4 - Fv) <= 1e-7 * abs(Fv) + 1e-9 * abs(dE)


@pytest.mark.parametrize("elem", ["hex", "wedge", "tet"])
def test_jacobian_complex_step(elem):
    m = _box_mesh(3, 3, 4, elem, seed=6)
    rng = np.random.default_rng(6)
    U = smooth_velocity(m, rng, 100.0, 0.05)
    _, J = fo.assemble(m, U)
    for picard in (False,):
        for _ in range(3):
            v = rng.normal(size=U.shape)
            h = 1e-30
            cs = fo.residual(m, U + 1j * h * v).imag / h
            Jv = J @ v
            assert np.abs(cs - Jv).max() <= 1e-12 * np.abs(Jv).max()


def test_jacobian_columns_central_fd():
    m = _box_mesh(2, 2, 2, "wedge", seed=7)
    U = smooth_velocity(m, np.random.default_rng(7), 100.0, 0.05)
    R, J = fo.assemble(m, U)
    Jd = J.toarray()
    h = 1e-4
    for j in range(m.n_dofs):
        e = np.zeros(m.n_dofs)
        e[j] = h
        col = (fo.residual(m, U + e) - fo.residual(m, U - e)) / (2 * h)
        scale = np.abs(Jd).max(axis=1) + 1e-300
        assert np.all(np.abs(col - Jd[:, j]) <= 1e-6 * scale)


def test_picard_part_drops_only_the_viscosity_derivative():
    m = _box_mesh(2, 2, 2, "hex", seed=8)
    U = smooth_velocity(m, np.random.default_rng(8), 100.0, 0.05)
    _, Jn = fo.assemble(m, U)
    _, Jp = fo.assemble(m, U, picard=True)
    D = (Jn - Jp).toarray()
    # the Newton part sum_q 2 mu' W g g^T is negative semidefinite for n > 1 (mu' < 0)
    w = np.linalg.eigvalsh(0.5 * (D + D.T))
    assert w.max() <= 1e-10 * np.abs(w).max()
    assert w.min() < 0
    # n = 1: no viscosity derivative, Newton == Picard
    m1 = m.with_fields(n=1.0)
    _, Jn1 = fo.assemble(m1, U)
    _, Jp1 = fo.assemble(m1, U, picard=True)
    assert abs(Jn1 - Jp1).max() == 0.0


# --------------------------------------------------------------------------------------
# P-6 / P-7: linearity for n = 1, homogeneity of degree 1/n
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("elem", ["hex", "wedge", "tet"])
def test_n1_residual_is_affine(elem):
    m = _box_mesh(3, 2, 3, elem, seed=9).with_fields(n=1.0)
    U = smooth_velocity(m, np.random.default_rng(9), 100.0, 0.05)
    R, J = fo.assemble(m, U)
    F0 = fo.residual(m, np.zeros_like(U))
    assert np.abs(R - (J @ U + F0)).max() <= 1e-12 * np.abs(R).max()


@pytest.mark.parametrize("n", [3.0, 2.0, 4.0])
def test_viscous_homogeneity(n):
    m = _box_mesh(3, 3, 2, "wedge", seed=10, beta=0.0).with_fields(n=n, eps0=0.0)
    U = smooth_velocity(m, np.random.default_rng(10), 100.0, 0.05)
    z = np.zeros(m.n_verts)
    F1 = fo.residual(m, U, s_drive=z)
    for lam in (0.5, 3.0):
        F2 = fo.residual(m, lam * U, s_drive=z)
        np.testing.assert_allclose(F2, lam ** (1.0 / n) * F1, rtol=0, atol=1e-12 * np.abs(F1).max())


# --------------------------------------------------------------------------------------
# pattern and ordering
# --------------------------------------------------------------------------------------

def test_pattern_count_slab():
    m, U = config0_slab()
    rowptr, colidx = fo.jacobian_pattern(m)
    L = m.n_layers
    # each vertex column owns 2 rows per level; a row couples D neighbouring columns
    # (itself included) on 2 or 3 levels
    D = np.zeros(m.n_verts, dtype=np.int64)
    for j in range(21):
        for i in range(21):
            nx = 3 - (i in (0, 20))
            ny = 3 - (j in (0, 20))
            D[j * 21 + i] = nx * ny
    assert rowptr[-1] == 238_144 == np.sum(4 * D * (3 * L + 1))
    R, J = fo.assemble(m, U)
    assert J.nnz == rowptr[-1]


def test_assemble_rows_matches_full():
    m = _box_mesh(4, 3, 3, "wedge", seed=11)
    U = smooth_velocity(m, np.random.default_rng(11), 100.0, 0.05)
    R, J = fo.assemble(m, U)
    sel = np.array([0, 5, 17, m.n_dofs - 1, m.n_dofs // 2])
    r, Jr, _ = fo.assemble_rows(m, U, sel)
    np.testing.assert_allclose(r, R[sel], rtol=1e-14, atol=0)
    assert abs(Jr - J[sel]).max() <= 1e-14 * abs(J).max()


# --------------------------------------------------------------------------------------
# tetrahedral extrusion: the split of each prism into three tetrahedra
# --------------------------------------------------------------------------------------

def test_chunked_assembly_keeps_the_prism_pattern():
    """Assembled in many chunks of cells, the tetrahedral Jacobian has the same pattern as in
    one chunk and as the wedge mesh (node pairs of a prism that share no tetrahedron stay as
    structural zeros) and the same values."""
    m = _box_mesh(6, 5, 3, "tet", seed=4)
    U = smooth_velocity(m, np.random.default_rng(2), 100.0, 0.05)
    _, J1 = fo.assemble(m, U)
    _, J7 = fo.assemble(m, U, chunk=7)
    _, Jw = fo.assemble(m.with_fields(elem="wedge"), U, chunk=5)
    for J in (J7, Jw):
        assert np.array_equal(J.indptr, J1.indptr) and np.array_equal(J.indices, J1.indices)
    assert (J1.data == 0).sum() > 0          # the structural zeros are there
    assert np.abs(J7.data - J1.data).max() <= 1e-13 * np.abs(J1.data).max()


def test_tet_split_is_conforming_and_fills_the_prisms():
    """Every triangular face of the tetrahedra is shared by exactly two of them or lies on
    the domain boundary (bed, surface, lateral sides), so neighbouring prisms split their
    common quad face along the same diagonal; the three tetrahedra of a prism with planar
    lower and upper faces fill it exactly."""
    m = _box_mesh(4, 3, 3, "tet", seed=12, pert=0.0)
    L = m.n_layers
    cells = np.arange(m.n_cells)
    tets = fo.tet_split(m, cells)                           # prism-local node indices
    nodes = fo.cell_nodes(m)[cells]
    glob = np.take_along_axis(nodes[:, None, :].repeat(3, axis=1), tets, axis=2).reshape(-1, 4)
    faces = {}
    for t in glob:
        for drop in range(4):
            f = tuple(sorted(np.delete(t, drop)))
            faces[f] = faces.get(f, 0) + 1
    assert max(faces.values()) == 2
    # faces seen once must lie on the boundary: all three nodes on the bed, on the surface,
    # or on one lateral side of the box
    xyz = fo.node_xyz(m)
    lev = np.tile(np.arange(L + 1), m.n_verts)
    xmax, ymax = m.xy[:, 0].max(), m.xy[:, 1].max()
    col_x = np.repeat(m.xy[:, 0], L + 1)
    col_y = np.repeat(m.xy[:, 1], L + 1)
    for f, c in faces.items():
        if c == 1:
            f = list(f)
            on = [np.all(lev[f] == 0), np.all(lev[f] == L), np.all(np.isclose(col_x[f], 0.0)),
                  np.all(np.isclose(col_x[f], xmax)), np.all(np.isclose(col_y[f], 0.0)),
                  np.all(np.isclose(col_y[f], ymax))]
            assert any(on), f
    # volumes: flat bed and surface, uniform H: every prism is a right prism
    flat = m.with_fields(thickness=np.full(m.n_verts, 600.0), surface=np.full(m.n_verts, 900.0))
    X = fo.node_xyz(flat)[nodes]
    _, vol, _ = fo._tet_geometry(X, tets)
    tri = m.xy[m.cells[cells // L]]
    area = 0.5 * np.abs((tri[:, 1, 0] - tri[:, 0, 0]) * (tri[:, 2, 1] - tri[:, 0, 1])
                        - (tri[:, 2, 0] - tri[:, 0, 0]) * (tri[:, 1, 1] - tri[:, 0, 1]))
    np.testing.assert_allclose(vol.sum(axis=1), area * 600.0 / L, rtol=1e-12)
