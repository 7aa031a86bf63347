"""Pins of the oracle's parity scales (no GPU).

Every GPU parity assertion divides by one of two oracle scales:
  * the per-term scale S (abs_terms / abs_scales): for each entry, the sum of the absolute
    values of every quadrature-point term summed into it; the rounding error of any
    summation order of those terms is at most a small multiple of the unit roundoff times S;
  * the element-level scale E (element_scales): sum over cells of |R_e,i|, and the row
    maximum of sum over cells of |J_e,ij|.
Here both are tied to facts that hold without them: they bound the entries they scale,
S equals the entry itself wherever every term has one sign (gravity load at U = 0, bed
friction under a uniform translation, the Picard diagonal), and on the Newton diagonal the
viscosity-derivative terms all have the opposite sign of the Picard terms, which fixes S
there exactly.  A dropped or mis-signed term in either scale fails one of these.
"""
import numpy as np
import pytest

from fo_inputs import config0_slab, perturbed, smooth_velocity, structured_box
from fo_inputs.meshgen import ExtrudedMesh
from oracle import fo_oracle as fo


def _box(elem, seed=0, nx=3, ny=2, L=2):
    xy, cells, sigma = structured_box(nx, ny, L, 4e3, 3e3, elem=elem)
    x, y = xy[:, 0], xy[:, 1]
    H = 800.0 + 100.0 * np.sin(2 * np.pi * x / 4e3) * np.cos(2 * np.pi * y / 3e3)
    m = ExtrudedMesh(elem, xy, cells, 500.0 - 0.01 * x + 0.004 * y + H, H, np.full(xy.shape[0], 900.0), sigma)
    m = perturbed(m, np.random.default_rng(seed), 0.25)
    return m, smooth_velocity(m, np.random.default_rng(seed), 80.0, 0.05)


def _sloped_cell(elem, sx, sy, beta=0.0):
    """One cell under a planar surface s = 300 + sx x + sy y with uniform thickness, so the
    bed is planar too and grad s is (sx, sy) at every point."""
    if elem == "hex":
        xy = np.array([[0.0, 0.0], [700.0, 0.0], [700.0, 400.0], [0.0, 400.0]])
        cells = np.array([[0, 1, 2, 3]], dtype=np.int32)
    else:
        xy = np.array([[0.0, 0.0], [600.0, 100.0], [150.0, 500.0]])
        cells = np.array([[0, 1, 2]], dtype=np.int32)
    H = np.full(xy.shape[0], 250.0)
    s = 300.0 + sx * xy[:, 0] + sy * xy[:, 1]
    return ExtrudedMesh(elem, xy, cells, s, H, np.full(xy.shape[0], beta), np.array([0.0, 1.0]))


CASES = {
    "box_hex": lambda: _box("hex", 1),
    "box_wedge": lambda: _box("wedge", 2),
    "slab_2000_hex": lambda: config0_slab(),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("picard", [False, True])
def test_scales_bound_the_entries(name, picard):
    """|R_i| <= E^R_i <= S^R_i, |J_ij| <= S^J_ij, and row maxima in the same order."""
    m, U = CASES[name]()
    R, J = fo.assemble(m, U, picard=picard)
    SR, SJ = fo.abs_terms(m, U, picard=picard)
    ER, EJ = fo.element_scales(m, U, picard=picard)
    rs, js = fo.abs_scales(m, U, picard=picard)
    slack = 1.0 + 1e-13
    assert np.all(np.abs(R) <= ER * slack)
    assert np.all(ER <= SR * slack)
    np.testing.assert_array_equal(rs, SR)
    # same pattern, every entry bounded
    assert np.array_equal(SJ.indptr, J.indptr) and np.array_equal(SJ.indices, J.indices)
    assert np.all(np.abs(J.data) <= SJ.data * slack)
    jmax = np.asarray(abs(J).max(axis=1).todense()).ravel()
    assert np.all(jmax <= EJ * slack)
    assert np.all(EJ <= js * slack)


@pytest.mark.parametrize("elem", ["hex", "wedge", "tet"])
def test_scale_equals_gravity_load_at_rest(elem):
    """U = 0 under a sloped planar surface: the strain rate vanishes, so each row of R is a
    sum of gravity terms W rho g (d_c s) N_a that all carry the sign of d_c s."""
    m = _sloped_cell(elem, -0.02, 0.006)
    U = np.zeros(m.n_dofs)
    R, _ = fo.assemble(m, U)
    SR, _ = fo.abs_terms(m, U)
    ER, _ = fo.element_scales(m, U)
    np.testing.assert_allclose(SR, np.abs(R), rtol=1e-15, atol=0)
    np.testing.assert_allclose(ER, np.abs(R), rtol=1e-15, atol=0)
    # and the load itself: rho g (d_c s) times the integral of N_a, i.e. the cell volume
    # split evenly over its nodes (linear basis in zeta, equal horizontal weights for the
    # box; for the wedge, every P1 triangle function integrates to area/3)
    vol = (700.0 * 400.0 if elem == "hex" else 0.5 * abs(600.0 * 500.0 - 150.0 * 100.0)) * 250.0
    rg = m.rho * m.g
    if elem == "tet":
        # the right prism splits into three tetrahedra of volume vol/3, each giving vol/12 to
        # its 4 nodes; the lowest-numbered base vertex is in 1 of them at the bed and 3 at the
        # top, the middle one in 2 and 2, the highest in 3 and 1
        share = np.zeros(6)
        order = np.argsort(m.cells[0])
        for cnt_b, cnt_t, corner in zip((1, 2, 3), (3, 2, 1), order):
            share[2 * corner] = cnt_b       # node v*(L+1) + 0 (bed), L = 1
            share[2 * corner + 1] = cnt_t   # node v*(L+1) + 1 (top)
        w = share * vol / 12.0
    else:
        w = np.full(m.n_dofs // 2, vol / (8 if elem == "hex" else 6))
    np.testing.assert_allclose(R[0::2], rg * -0.02 * w, rtol=1e-12)
    np.testing.assert_allclose(R[1::2], rg * 0.006 * w, rtol=1e-12)


@pytest.mark.parametrize("elem", ["hex", "wedge", "tet"])
def test_scale_equals_bed_friction_under_translation(elem):
    """Flat surface, uniform velocity (c1, c2) with c1, c2 > 0: no strain rate, no gravity,
    each row is a sum of bed terms W beta c_c N_a N_b >= 0.  (The strain rate of a uniform
    field is zero only up to rounding, ~1e-17 /yr, where the regularised viscosity is ~1e12:
    those viscous terms come to ~1e-9 of the bed terms, hence the tolerance.)"""
    m = _sloped_cell(elem, 0.0, 0.0, beta=700.0)
    U = np.tile([30.0, 12.0], m.n_dofs // 2)
    R, _ = fo.assemble(m, U)
    SR, _ = fo.abs_terms(m, U)
    bed_rows = np.zeros(m.n_dofs, dtype=bool)
    bed_rows[0::4] = bed_rows[1::4] = True          # node v*(L+1) + 0, L = 1
    np.testing.assert_allclose(SR[bed_rows], R[bed_rows], rtol=1e-8)
    assert np.all(SR[~bed_rows] <= 1e-8 * SR[bed_rows].max())   # upper rows: zero up to rounding
    # the bed term integrates beta c_c N_a over the (flat) lower face: beta c_c area / nv
    area = 700.0 * 400.0 if elem == "hex" else 0.5 * abs(600.0 * 500.0 - 150.0 * 100.0)
    nv = 4 if elem == "hex" else 3
    np.testing.assert_allclose(R[0::4], 700.0 * 30.0 * area / nv, rtol=1e-8)
    np.testing.assert_allclose(R[1::4], 700.0 * 12.0 * area / nv, rtol=1e-8)


@pytest.mark.parametrize("name", ["box_hex", "box_wedge"])
def test_diagonal_scales_pin_picard_and_newton_terms(name):
    """On the diagonal every Picard term (2 mu W K_cc(grad N_a, grad N_a), bed mass) is
    >= 0 and, for n > 1, every viscosity-derivative term 2 mu' W g^2 is <= 0.  So
    S^J_ii = J^P_ii for the Picard Jacobian, and S^J_ii = 2 J^P_ii - J_ii for Newton's."""
    m, U = CASES[name]()
    assert m.n > 1
    _, JP = fo.assemble(m, U, picard=True)
    _, JN = fo.assemble(m, U, picard=False)
    _, SP = fo.abs_terms(m, U, picard=True)
    _, SN = fo.abs_terms(m, U, picard=False)
    dP, dN = JP.diagonal(), JN.diagonal()
    np.testing.assert_allclose(SP.diagonal(), dP, rtol=1e-13)
    np.testing.assert_allclose(SN.diagonal(), 2 * dP - dN, rtol=1e-12)
    assert np.all(dN < dP)       # the derivative term lowers every diagonal entry


def test_per_term_scale_against_element_scale_on_slab():
    """How much looser the per-term scale is than the element-level one on the 2000-hex
    slab with its seeded velocity: residual rows up to 290x (median 1.41x; rows where the
    viscous and gravity terms of one element cancel), Jacobian rows up to 4x.  Norm-wise
    the per-term residual scale stays within 1.6 ||R||_inf."""
    m, U = config0_slab()
    R, _ = fo.assemble(m, U)
    rs, js = fo.abs_scales(m, U)
    er, ej = fo.element_scales(m, U)
    ratio_r, ratio_j = rs / er, js / ej
    assert 200.0 < ratio_r.max() <= 300.0
    assert 1.3 < np.median(ratio_r) < 1.5
    assert 3.5 < ratio_j.max() <= 4.1
    assert rs.max() <= 1.6 * np.abs(R).max()
