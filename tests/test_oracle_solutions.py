"""Solution-level pins of the oracle: an exact slab solution, a manufactured smooth
solution with mesh refinement, and the shallow-ice initial guess (no GPU)."""
import numpy as np
import pytest

from fo_inputs import structured_box
from fo_inputs.meshgen import ExtrudedMesh
from oracle import fo_oracle as fo
from oracle import solve

RG = 910.0 * 9.81


# --------------------------------------------------------------------------------------
# P-8: parallel slab on a flat bed driven by a surface slope: v = 0 and
# u(z) = rho g H tan(a) / beta + 2 A (rho g tan a)^n [H^(n+1) - (H - z)^(n+1)] / (n + 1)
# --------------------------------------------------------------------------------------

def _slab(L, elem, H=1000.0, beta=1000.0, alpha_deg=0.5):
    xy, cells, sigma = structured_box(1, 1, L, 2e3, 2e3, elem=elem)
    V = xy.shape[0]
    m = ExtrudedMesh(elem, xy, cells, np.full(V, H), np.full(V, H), np.full(V, beta), sigma)
    ta = np.tan(np.deg2rad(alpha_deg))
    s_drive = H - xy[:, 0] * ta
    return m, s_drive, ta


def _slab_exact(m, ta, H=1000.0, beta=1000.0):
    z = fo.node_xyz(m)[:, 2]
    n, A = m.n, m.A
    u = RG * H * ta / beta + 2 * A * (RG * ta) ** n * (H ** (n + 1) - (H - z) ** (n + 1)) / (n + 1)
    return np.stack([u, np.zeros_like(u)], axis=1).reshape(-1)


@pytest.mark.parametrize("elem", ["hex", "wedge"])
def test_exact_slab_second_order(elem):
    errs = []
    for L in (4, 8, 16, 32):
        m, s_drive, ta = _slab(L, elem)
        ex = _slab_exact(m, ta)
        U0 = np.zeros(m.n_dofs)
        U0[0::2] = 80.0
        U, info = solve.newton_solve(m, U0, tol=1e-10, s_drive=s_drive)
        assert info["status"] == "converged", info
        errs.append(np.abs(U - ex).max() / np.abs(ex).max())
        assert np.abs(U[1::2]).max() < 1e-9          # no cross-flow
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert np.all(rates > 1.9), (errs, rates)
    assert errs[-1] < 2e-4
    # surface speed by hand: rho g H tan(0.5 deg) / beta = 77.90 m/yr of sliding plus
    # A (rho g tan 0.5 deg)^3 H^4 / 2 = 23.64 m/yr of shear
    assert abs(ex[-2] - 101.5) < 0.5


def test_exact_slab_tetrahedra_first_order():
    """The same slab on tetrahedra (3 per prism): P1 on the split prism is not exact for the
    vertical profile, and the slanted faces turn part of the vertical shear into spurious
    horizontal strain (cross-flow v), so nodal errors and cross-flow fall at first order as
    the layers are refined (the oracle's split and P1 gradients are what make them vanish)."""
    errs, cross = [], []
    for L in (4, 8, 16, 32):
        m, s_drive, ta = _slab(L, "tet")
        ex = _slab_exact(m, ta)
        U0 = np.zeros(m.n_dofs)
        U0[0::2] = 80.0
        U, info = solve.newton_solve(m, U0, tol=1e-10, s_drive=s_drive)
        assert info["status"] == "converged", info
        errs.append(np.abs(U - ex).max() / np.abs(ex).max())
        cross.append(np.abs(U[1::2]).max() / np.abs(ex).max())
    errs, cross = np.array(errs), np.array(cross)
    rates = np.log2(errs[:-1] / errs[1:])
    crates = np.log2(cross[:-1] / cross[1:])
    assert np.all(rates > 0.95) and np.all(crates > 0.95), (errs, rates, cross, crates)
    assert errs[-1] < 4e-3 and cross[-1] < 3e-3


# --------------------------------------------------------------------------------------
# P-9: manufactured smooth solution, non-flat bed and surface, n = 3 with eps0,
# lateral Dirichlet columns, volume source and top/bed tractions from the exact field
# --------------------------------------------------------------------------------------

LX = LY = 10e3
KX, KY = np.pi / LX, np.pi / LY


def _geom(x, y):
    b = 100.0 * np.sin(KX * x) * np.sin(KY * y)
    H = 800.0 + 150.0 * np.cos(KX * x) * np.cos(KY * y)
    bx = 100.0 * KX * np.cos(KX * x) * np.sin(KY * y)
    by = 100.0 * KY * np.sin(KX * x) * np.cos(KY * y)
    Hx = -150.0 * KX * np.sin(KX * x) * np.cos(KY * y)
    Hy = -150.0 * KY * np.cos(KX * x) * np.sin(KY * y)
    return b, H, bx, by, bx + Hx, by + Hy


def _beta(x, y):
    return 500.0 * (1.0 + 0.5 * np.sin(KX * x) * np.sin(KY * y))


def _exact(x, y, z):
    sx, cx, sy, cy = np.sin(KX * x), np.cos(KX * x), np.sin(KY * y), np.cos(KY * y)
    u = 40 + 15 * sx * cy + 0.02 * z + 2e-5 * z ** 2
    v = 10 * cx * sy + 0.01 * z - 1e-5 * z ** 2
    ux, uy, uz = 15 * KX * cx * cy, -15 * KY * sx * sy, 0.02 + 4e-5 * z
    vx, vy, vz = -10 * KX * sx * sy, 10 * KY * cx * cy, 0.01 - 2e-5 * z
    return u, v, (ux, uy, uz, vx, vy, vz)


def _fluxes(x, y, z, A=1e-16, n=3.0, eps0=1e-10):
    _, _, (ux, uy, uz, vx, vy, vz) = _exact(x, y, z)
    exx, eyy, exy, exz, eyz = ux, vy, 0.5 * (uy + vx), 0.5 * uz, 0.5 * vz
    q = exx ** 2 + eyy ** 2 + exx * eyy + exy ** 2 + exz ** 2 + eyz ** 2
    mu = 0.5 * A ** (-1 / n) * (q + eps0 ** 2) ** ((1 - n) / (2 * n))
    f1 = 2 * mu[..., None] * np.stack([2 * exx + eyy, exy, exz], axis=-1)
    f2 = 2 * mu[..., None] * np.stack([exy, exx + 2 * eyy, eyz], axis=-1)
    return f1, f2


def _source(p):
    """f_c = -div(2 mu eps_c) + rho g d_c s, divergence by 4th-order differences."""
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    div = [np.zeros_like(x), np.zeros_like(x)]
    for d, h in ((0, 1.0), (1, 1.0), (2, 0.1)):
        off = np.zeros(3)
        off[d] = h
        acc = [np.zeros_like(x), np.zeros_like(x)]
        for k, w in ((1, 8.0), (2, -1.0)):
            fp = _fluxes(x + k * off[0], y + k * off[1], z + k * off[2])
            fm = _fluxes(x - k * off[0], y - k * off[1], z - k * off[2])
            for c in range(2):
                acc[c] += w * (fp[c][..., d] - fm[c][..., d])
        for c in range(2):
            div[c] += acc[c] / (12 * h)
    _, _, _, _, s_x, s_y = _geom(x, y)
    return np.stack([-div[0] + RG * s_x, -div[1] + RG * s_y], axis=-1)


def _mms_hooks(mesh):
    ref = fo.RefElement(mesh.elem)
    tpts = ref.bpts.copy()
    tpts[:, 2] = 1.0
    Nt, dNt = ref._basis(tpts)
    L = mesh.n_layers

    def face(X, N, dN, w):
        tx = np.einsum("cai,ra->cri", X, dN[..., 0])
        ty = np.einsum("cai,ra->cri", X, dN[..., 1])
        nrm = np.cross(tx, ty)
        dA = w[None, :] * np.linalg.norm(nrm, axis=-1)
        p = np.einsum("ra,cai->cri", N, X)
        return p, dA

    def hooks(m, ref_, cell_ids, nodes, X, Ue, gradN, W, Re, Je):
        xq = np.einsum("qa,cai->cqi", ref_.N, X)
        f = _source(xq)
        Re -= np.einsum("cq,cqk,qa->cak", W, f, ref_.N)
        layer = cell_ids % L
        for sel, N, dN, w, top in ((layer == 0, ref_.Nb, ref_.dNb, ref_.bw, False),
                                   (layer == L - 1, Nt, dNt, ref_.bw, True)):
            if not np.any(sel):
                continue
            idx = np.nonzero(sel)[0]
            p, dA = face(X[idx], N, dN, w)
            x, y, z = p[..., 0], p[..., 1], p[..., 2]
            _, _, bx, by, sx, sy = _geom(x, y)
            if top:
                nv = np.stack([-sx, -sy, np.ones_like(sx)], axis=-1)
            else:
                nv = np.stack([bx, by, -np.ones_like(bx)], axis=-1)
            nv /= np.linalg.norm(nv, axis=-1, keepdims=True)
            f1, f2 = _fluxes(x, y, z)
            h = np.stack([np.sum(f1 * nv, -1), np.sum(f2 * nv, -1)], axis=-1)
            if not top:
                u, v, _ = _exact(x, y, z)
                h = h + _beta(x, y)[..., None] * np.stack([u, v], axis=-1)
            Re[idx] -= np.einsum("cr,crk,ra->cak", dA, h, N)

    return hooks


def _mms_mesh(nb, L, elem):
    xy, cells, sigma = structured_box(nb, nb, L, LX, LY, elem=elem)
    b, H, *_ = _geom(xy[:, 0], xy[:, 1])
    return ExtrudedMesh(elem, xy, cells, b + H, H, _beta(xy[:, 0], xy[:, 1]), sigma)


@pytest.mark.parametrize("elem", ["hex", "wedge"])
def test_manufactured_solution_refinement(elem):
    errs = []
    for nb in (4, 8, 16):
        m = _mms_mesh(nb, nb // 2, elem)
        xyz = fo.node_xyz(m)
        u, v, _ = _exact(xyz[:, 0], xyz[:, 1], xyz[:, 2])
        ex = np.stack([u, v], axis=1).reshape(-1)
        on_bnd = ((np.isclose(m.xy[:, 0], 0) | np.isclose(m.xy[:, 0], LX)
                   | np.isclose(m.xy[:, 1], 0) | np.isclose(m.xy[:, 1], LY)))
        fixed_nodes = np.repeat(on_bnd, m.n_layers + 1)
        fixed = np.repeat(fixed_nodes, 2)
        U0 = ex * (1 + 0.05 * np.random.default_rng(nb).normal(size=ex.shape))
        U0[fixed] = ex[fixed]
        U, info = solve.newton_solve(m, U0, tol=1e-10, fixed=fixed, fixed_values=ex,
                                     hooks=_mms_hooks(m))
        assert info["status"] == "converged", info
        free = ~fixed
        errs.append(np.sqrt(np.mean((U[free] - ex[free]) ** 2)) / np.sqrt(np.mean(ex[free] ** 2)))
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert np.all(rates > 1.7), (errs, rates)


# --------------------------------------------------------------------------------------
# shallow-ice initial guess
# --------------------------------------------------------------------------------------

def test_sia_matches_closed_form_on_planar_slab():
    xy, cells, sigma = structured_box(6, 5, 7, 6e3, 5e3, elem="wedge")
    rng = np.random.default_rng(3)
    xy[:, :] += rng.uniform(-150, 150, xy.shape) * (
        (xy[:, :1] > 0) & (xy[:, :1] < 6e3) & (xy[:, 1:] > 0) & (xy[:, 1:] < 5e3))
    ta = np.tan(np.deg2rad(0.7))
    H = np.full(xy.shape[0], 1200.0)
    s = 2000.0 - ta * xy[:, 0] + 0.3 * ta * xy[:, 1]
    beta = np.full(xy.shape[0], 800.0)
    m = ExtrudedMesh("wedge", xy, cells, s, H, beta, sigma)
    gx, gy = solve.vertex_surface_gradient(m)
    np.testing.assert_allclose(gx, -ta, rtol=1e-10)
    np.testing.assert_allclose(gy, 0.3 * ta, rtol=1e-10)
    U = solve.sia_guess(m).reshape(-1, 2)
    gm = ta * np.sqrt(1 + 0.09)
    z = fo.node_xyz(m)[:, 2]
    zb = np.repeat(s - H, m.n_layers + 1)
    speed = RG * 1200.0 * gm / 800.0 + 2 * m.A / 4 * RG ** 3 * gm ** 3 * (
        1200.0 ** 4 - (1200.0 - (z - zb)) ** 4)
    np.testing.assert_allclose(np.hypot(U[:, 0], U[:, 1]), speed, rtol=1e-10)
    # flow is down the surface gradient
    np.testing.assert_allclose(U[:, 1] / U[:, 0], -0.3, rtol=1e-10)


def test_sia_quad_gradient_and_cap():
    xy, cells, sigma = structured_box(4, 4, 3, 4e3, 4e3, elem="hex")
    s = 1500.0 + 0.01 * xy[:, 0] - 0.02 * xy[:, 1]
    H = np.full(xy.shape[0], 900.0)
    beta = np.full(xy.shape[0], 1e-9)       # nearly free slip: sliding speed capped
    m = ExtrudedMesh("hex", xy, cells, s, H, beta, sigma)
    gx, gy = solve.vertex_surface_gradient(m)
    np.testing.assert_allclose(gx, 0.01, rtol=1e-12)
    np.testing.assert_allclose(gy, -0.02, rtol=1e-12)
    U = solve.sia_guess(m).reshape(-1, 2, )
    base = U.reshape(m.n_verts, m.n_layers + 1, 2)[:, 0, :]
    np.testing.assert_allclose(np.hypot(base[:, 0], base[:, 1]), 1e4, rtol=1e-12)
