"""Pins of the oracle's ocean back-pressure term on marked lateral fronts (no GPU).

Reading of the lateral condition of Sec. 2: 2 mu eps_i . n - rho g (s - z) n_i =
-rho_w g max(-z, 0) n_i on the marked fronts, sea level at z = 0, so the residual gains
-int phi_a p(z) n_i dA with p = rho g (s - z) - rho_w g max(-z, 0).

The nodal loads of each face are pinned by moments computed without the face basis: the
face lies in the vertical plane of its edge, a planar quadrilateral in (arc length, z); its
parts above and below sea level are cut out as polygons and the moments of p times
1, arc length and z integrated exactly on triangles (degree-2 midpoint rule).  The bilinear
face basis reproduces 1, arc length and z, so the sums of the loads weighted by those nodal
values must equal the polygon moments.  A freely floating slab gives the classic front force
1/2 rho g H^2 (1 - rho/rho_w) per unit width, and the depth-summed residual of its biaxial
spreading field vanishes column by column.
"""
import numpy as np
import pytest

from fo_inputs import floating_slab, marine_sheet
from oracle import fo_oracle as fo


def _clip(poly, keep_below):
    """Sutherland-Hodgman clip of a polygon [(t, z)] to z <= 0 (or z >= 0)."""
    sgn = 1.0 if keep_below else -1.0
    out = []
    for i in range(len(poly)):
        p, q = poly[i], poly[(i + 1) % len(poly)]
        fp, fq = sgn * p[1], sgn * q[1]
        if fp <= 0:
            out.append(p)
        if (fp < 0 < fq) or (fq < 0 < fp):
            r = fp / (fp - fq)
            out.append((p[0] + r * (q[0] - p[0]), p[1] + r * (q[1] - p[1])))
    return out


def _poly_integral(poly, f):
    """Exact integral of a quadratic f(t, z) over a convex polygon (fan of triangles, each by
    the edge-midpoint rule, exact to degree 2)."""
    tot = 0.0
    for i in range(1, len(poly) - 1):
        a, b, c = np.array(poly[0]), np.array(poly[i]), np.array(poly[i + 1])
        area = 0.5 * abs((b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]))
        mids = [(a + b) / 2, (b + c) / 2, (c + a) / 2]
        tot += area / 3.0 * sum(f(m[0], m[1]) for m in mids)
    return tot


def _face_moments(m, length, zc, sab):
    """int p * (1, t, z) dA over one face, t the arc length from the face's first corner."""
    rg, rwg = m.rho * m.g, m.rho_w * m.g
    poly = [(0.0, zc[0]), (length, zc[1]), (length, zc[2]), (0.0, zc[3])]
    s_of = lambda t: sab[0] + (sab[1] - sab[0]) * t / length
    out = np.zeros(3)
    for below in (True, False):
        part = _clip(poly, below)
        if len(part) < 3:
            continue
        water = rwg if below else 0.0
        p = lambda t, z: rg * (s_of(t) - z) + water * z      # -rho_w g max(-z, 0) = rho_w g z below
        for j, w in enumerate((lambda t, z: 1.0, lambda t, z: t, lambda t, z: z)):
            out[j] += _poly_integral(part, lambda t, z: p(t, z) * w(t, z))
    return out


@pytest.mark.parametrize("which", ["slab_hex", "slab_wedge_jitter", "steep", "marine"])
def test_face_loads_match_polygon_moments(which):
    if which == "slab_hex":
        m = floating_slab("hex")
    elif which == "steep":
        # thickness alternating 40 m / 2000 m along the fronts: layer thicknesses differ 50x
        # between the two ends of a face (the water term's pole sits just outside it)
        m = floating_slab("hex", nx=5, ny=4, n_layers=4)
        H = np.where((np.round(m.xy[:, 0] / 6e3) + np.round(m.xy[:, 1] / 5e3)) % 2 == 0, 40.0, 2000.0)
        m = m.with_fields(thickness=H, surface=(1 - m.rho / m.rho_w) * H)
    elif which == "slab_wedge_jitter":
        m = floating_slab("wedge", jitter=0.25, seed=3)
        m = m.with_fields(thickness=m.thickness * (1 + 0.3 * np.sin(m.xy[:, 0] / 7e3)),
                          surface=m.surface + 25 * np.cos(m.xy[:, 1] / 5e3))
    else:
        m, _ = marine_sheet(seed=2, n_points=400, n_layers=4)
    nodes, normal, length, zc, sab = fo.front_faces(m)
    fn, tot, _ = fo.front_face_terms(m)
    assert np.array_equal(fn, nodes)
    t_nodes = np.stack([np.zeros_like(length), length, length, np.zeros_like(length)], axis=1)
    crossing = 0
    for f in range(nodes.shape[0]):
        mom = _face_moments(m, length[f], zc[f], sab[f])
        crossing += int(zc[f].min() < 0 < zc[f].max())
        for c in range(2):
            got = np.array([tot[f, :, c].sum(), (tot[f, :, c] * t_nodes[f]).sum(), (tot[f, :, c] * zc[f]).sum()])
            want = -normal[f, c] * mom
            scale = np.abs(normal[f, c]) * np.array([1.0, length[f], np.abs(zc[f]).max()]) * \
                abs(m.rho * m.g) * length[f] * np.ptp(zc[f]) * (np.abs(zc[f]).max() + np.abs(sab[f]).max())
            assert np.all(np.abs(got - want) <= 1e-12 * scale + 1e-300), (which, f, c, got, want)
    assert crossing > 0     # some faces straddle the sea level


def test_floating_slab_front_force_and_spreading_balance():
    """Uniform floating slab, every side a front: the load on one front is
    -1/2 rho g H^2 (1 - rho/rho_w) per unit width along its normal, and at the biaxial
    spreading field u = a (x - xc), v = a (y - yc) with
    a = A [rho g H (1 - rho/rho_w) / (6 * 3^((1-n)/(2n)))]^n the residual summed over each
    vertex column vanishes (the depth-integrated membrane stress balances the front force)."""
    for elem in ("hex", "wedge"):
        m = floating_slab(elem, nx=5, ny=4, n_layers=3, lx=25e3, ly=16e3, H=500.0)
        m = m.with_fields(eps0=0.0)
        H, rho, rw, g, n, A = 500.0, m.rho, m.rho_w, m.g, m.n, m.A
        L1 = m.n_layers + 1
        Fl = fo.front_load(m).reshape(-1, L1, 2)
        right = np.isclose(m.xy[:, 0], 25e3)
        force = 0.5 * rho * g * H ** 2 * (1 - rho / rw)
        assert abs(Fl[right, :, 0].sum() + force * 16e3) <= 1e-13 * force * 16e3
        assert abs(Fl[right, :, 1].sum()) <= 1e-13 * force * 16e3
        a = A * (rho * g * H * (1 - rho / rw) / (6.0 * 3.0 ** ((1 - n) / (2 * n)))) ** n
        xc, yc = 12.5e3, 8e3
        U = np.zeros((m.n_verts, L1, 2))
        U[:, :, 0] = a * (m.xy[:, 0] - xc)[:, None]
        U[:, :, 1] = a * (m.xy[:, 1] - yc)[:, None]
        R = fo.residual(m, U.reshape(-1)).reshape(-1, L1, 2)
        col = R.sum(axis=1)
        scale = np.abs(fo.front_load(m, absolute=True)).reshape(-1, L1, 2).sum(axis=1).max()
        assert np.abs(col).max() <= 1e-13 * scale, np.abs(col).max() / scale
        # node by node it does not vanish: the load varies with depth, the stress does not
        assert np.abs(R).max() > 1e-3 * scale


def test_front_rejects_interior_edges():
    m = floating_slab("wedge")
    interior = np.array([[m.cells[0, 0], m.cells[0, 2]]])     # the diagonal of the first quad
    with pytest.raises(ValueError):
        fo.front_faces(m.with_fields(front_edges=interior))


def test_front_term_does_not_change_the_jacobian():
    """The front load does not depend on U: the complex-step derivative of the residual with
    fronts equals the analytic Jacobian (which has no front term)."""
    m, U = marine_sheet(seed=4, n_points=120, n_layers=2)
    R, J = fo.assemble(m, U)
    rng = np.random.default_rng(0)
    v = rng.normal(size=m.n_dofs)
    h = 1e-30 * np.abs(U).max()
    Jv_cs = fo.residual(m, U + 1j * h * v).imag / h
    assert np.abs(J @ v - Jv_cs).max() <= 1e-10 * np.abs(J @ v).max()
    m0 = m.with_fields(front_edges=None)
    assert np.allclose(R - fo.residual(m0, U), fo.front_load(m), rtol=0, atol=1e-9 * np.abs(R).max())
