"""FP64 CPU oracle for first-order (Blatter-Pattyn) Stokes finite-element assembly.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product library never does.
It shares no code with the HIP path: it takes the seeded input arrays and
evaluates the textbook definitions directly, cell by cell and quadrature point
by quadrature point, vectorised over chunks of cells with NumPy, summing
element contributions into a SciPy CSR matrix.

What it computes (arXiv:2204.04321):
  * Sec. 2, eq. (FOStokes): -div(2 mu eps1) + rho g ds/dx = 0,
    -div(2 mu eps2) + rho g ds/dy = 0, with the strain-rate vectors eps1, eps2
    and components eps_xx = u_x, eps_yy = v_y, eps_xy = (u_y + v_x)/2,
    eps_xz = u_z/2, eps_yz = v_z/2 defined right after it;
  * eq. (effvisc): mu = 1/2 A^(-1/n) eps_e^(1/n - 1), here with the regularised
    form 1/2 A^(-1/n) (eps_e^2 + eps0^2)^((1-n)/(2n)) (reading: eps0 = 1e-10/yr);
  * eq. (effeps): eps_e^2 = eps_xx^2 + eps_yy^2 + eps_xx eps_yy + eps_xy^2
    + eps_xz^2 + eps_yz^2;
  * Sec. 2 boundary conditions: stress-free upper surface (natural), linear
    sliding 2 mu eps_i . n + beta u_i = 0 on the bed (reading: "= 0" is implied),
    lateral margin natural (no term) except on the marked ocean fronts, where the
    lateral condition of Sec. 2 applies, read as 2 mu eps_i . n - rho g (s - z) n_i
    = -rho_w g max(-z, 0) n_i with sea level z = 0 (the printed max(z, 0) and its sign
    are garbled: water pushes on the submerged part, against the outward normal);
  * Sec. 3.1, eq. (residual): the discrete residual F(U) assembled from nodal
    basis functions phi_i and their gradients on prismatic (wedge) or
    hexahedral elements extruded from the 2D mesh;
  * eq. (linearsystem): the Jacobian J = dF/dU, formed here analytically by
    differentiating the integrand by hand (the GPU path uses forward-mode AD,
    Sec. 3.2, so the two are computed independently).

Weak form used (test function phi_a, component c in {x, y}):
  F_(a,c) = sum_cells sum_q W_q [2 mu eps_c . grad phi_a + rho g (d_c s) phi_a]
          + sum_bed_faces sum_r W^b_r beta_r u_c(r) phi_a(r)
Readings where the paper is silent: the surface gradient d_c s is the
interpolant of nodal s differentiated with the 3D basis gradients; quadrature
is 2x2x2 Gauss (hex) and the 3-point degree-2 triangle rule x 2-point Gauss
(wedge); the bed measure is the physical 3D face area; reference coordinates
lie in [0,1]; node elevations are z = (s - H) + sigma_k H with vertical columns.

Tetrahedral extrusion (elem "tet", the element of the paper's nightly test, Sec. 5.3:
3 tetrahedra per layer and base triangle): each prism is split by the global order of
its base vertices p0 < p1 < p2 into (p0, p1, p2, p0'), (p1, p2, p0', p1'), (p2, p0', p1', p2')
(primes: one level up), so the diagonal of every lateral quad face runs from the bottom of
its higher-numbered vertex to the top of its lower-numbered one and neighbouring prisms
agree.  Linear (P1) basis on each tetrahedron: gradients, strain rate and viscosity are
constant in it, so its integrals are exact without quadrature (int phi_a = V/4).  The bed
term is the prism's (its lower face is the first tetrahedron's face, where the P1 basis is
the triangle's).  The CSR pattern stays the prism's: node pairs of a prism that share no
tetrahedron are structural zeros.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# --------------------------------------------------------------------------------------
# reference elements
# --------------------------------------------------------------------------------------

_G1 = 0.5 - 0.5 / np.sqrt(3.0)
_G2 = 0.5 + 0.5 / np.sqrt(3.0)


class RefElement:
    """Basis values/derivatives on the reference cell at volume and bed quadrature points."""

    def __init__(self, elem: str):
        self.elem = elem
        if elem == "wedge":
            tri = [(1 / 6, 1 / 6), (2 / 3, 1 / 6), (1 / 6, 2 / 3)]
            pts, wts = [], []
            for zq in (_G1, _G2):
                for (xq, yq) in tri:
                    pts.append((xq, yq, zq))
                    wts.append((1 / 6) * 0.5)
            bpts = [(xq, yq, 0.0) for (xq, yq) in tri]
            bwts = [1 / 6] * 3
            self.nv = 3
        elif elem == "hex":
            pts, wts = [], []
            for zq in (_G1, _G2):
                for yq in (_G1, _G2):
                    for xq in (_G1, _G2):
                        pts.append((xq, yq, zq))
                        wts.append(0.125)
            bpts = [(xq, yq, 0.0) for yq in (_G1, _G2) for xq in (_G1, _G2)]
            bwts = [0.25] * 4
            self.nv = 4
        else:
            raise ValueError(elem)
        self.npe = 2 * self.nv
        self.pts = np.array(pts)
        self.w = np.array(wts)
        self.bpts = np.array(bpts)
        self.bw = np.array(bwts)
        self.N, self.dN = self._basis(self.pts)
        self.Nb, self.dNb = self._basis(self.bpts)

    def _basis2d(self, xi, eta):
        if self.elem == "wedge":
            lam = np.array([1 - xi - eta, xi, eta])
            dlam = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
        else:
            lam = np.array([(1 - xi) * (1 - eta), xi * (1 - eta), xi * eta, (1 - xi) * eta])
            dlam = np.array([[-(1 - eta), -(1 - xi)], [(1 - eta), -xi], [eta, xi], [-eta, (1 - xi)]])
        return lam, dlam

    def _basis(self, pts):
        nq = pts.shape[0]
        N = np.zeros((nq, self.npe))
        dN = np.zeros((nq, self.npe, 3))
        for q, (xi, eta, zeta) in enumerate(pts):
            lam, dlam = self._basis2d(xi, eta)
            ell = np.array([1 - zeta, zeta])
            dell = np.array([-1.0, 1.0])
            for lev in range(2):
                for i in range(self.nv):
                    a = lev * self.nv + i
                    N[q, a] = lam[i] * ell[lev]
                    dN[q, a, 0] = dlam[i, 0] * ell[lev]
                    dN[q, a, 1] = dlam[i, 1] * ell[lev]
                    dN[q, a, 2] = lam[i] * dell[lev]
        return N, dN


# --------------------------------------------------------------------------------------
# mesh helpers
# --------------------------------------------------------------------------------------

def cell_nodes(mesh) -> np.ndarray:
    """Global node ids [n_cells, npe]; cell index = base_cell * L + layer; local nodes:
    the base cell's vertices at the lower level, then the same vertices one level up."""
    L = mesh.n_layers
    base = mesh.cells.astype(np.int64)
    k = np.arange(L, dtype=np.int64)
    bottom = base[:, None, :] * (L + 1) + k[None, :, None]
    return np.concatenate([bottom, bottom + 1], axis=2).reshape(-1, base.shape[1] * 2)


def node_xyz(mesh) -> np.ndarray:
    L1 = mesh.n_layers + 1
    bed = mesh.surface - mesh.thickness
    z = bed[:, None] + mesh.sigma[None, :] * mesh.thickness[:, None]
    xyz = np.empty((mesh.n_verts, L1, 3))
    xyz[:, :, 0] = mesh.xy[:, 0][:, None]
    xyz[:, :, 1] = mesh.xy[:, 1][:, None]
    xyz[:, :, 2] = z
    return xyz.reshape(-1, 3)


def node_column_field(mesh, f: np.ndarray) -> np.ndarray:
    """Extend a per-vertex field to every node of the vertex column."""
    return np.repeat(f, mesh.n_layers + 1)


# --------------------------------------------------------------------------------------
# element-level evaluation
# --------------------------------------------------------------------------------------

def _local(X: np.ndarray) -> np.ndarray:
    """Cell node coordinates relative to the cell's first node.  The derivatives of the
    isoparametric map do not change under a translation of the cell (the basis derivatives
    sum to zero), and the differences of coordinates of ~1e6 m are exact here, so this only
    removes the rounding of the map's Jacobian entries formed from large absolute
    coordinates (about 1e-16 x 1e6 m on a 5 m-thick margin cell)."""
    return X - X[:, :1, :]


def _geometry(ref: RefElement, X: np.ndarray):
    """X [nc, npe, 3] -> (gradN [nc,nq,npe,3], W [nc,nq]) by the isoparametric map."""
    Jm = np.einsum("cai,qaj->cqij", _local(X), ref.dN)  # dx_i / dxi_j
    det = np.linalg.det(Jm)
    inv = np.linalg.inv(Jm)                              # dxi_j / dx_i  (index [j, i])
    gradN = np.einsum("qaj,cqji->cqai", ref.dN, inv)
    W = ref.w[None, :] * det
    return gradN, W, det


def _strain(gradN, Ue):
    """Velocity gradients at the quadrature points and the strain-rate components."""
    u = Ue[:, :, 0]
    v = Ue[:, :, 1]
    ux = np.einsum("ca,cqa->cq", u, gradN[..., 0])
    uy = np.einsum("ca,cqa->cq", u, gradN[..., 1])
    uz = np.einsum("ca,cqa->cq", u, gradN[..., 2])
    vx = np.einsum("ca,cqa->cq", v, gradN[..., 0])
    vy = np.einsum("ca,cqa->cq", v, gradN[..., 1])
    vz = np.einsum("ca,cqa->cq", v, gradN[..., 2])
    exx, eyy = ux, vy
    exy = 0.5 * (uy + vx)
    exz = 0.5 * uz
    eyz = 0.5 * vz
    return exx, eyy, exy, exz, eyz


def effective_strain_rate_sq(exx, eyy, exy, exz, eyz):
    """eq. (effeps)."""
    return exx ** 2 + eyy ** 2 + exx * eyy + exy ** 2 + exz ** 2 + eyz ** 2


def viscosity(q, A, n, eps0):
    """eq. (effvisc) with regularisation: mu and d mu / d(eps_e^2)."""
    qe = q + eps0 ** 2
    mu = 0.5 * A ** (-1.0 / n) * qe ** ((1.0 - n) / (2.0 * n))
    dmu = ((1.0 - n) / (2.0 * n)) * mu / qe
    return mu, dmu


def tet_split(mesh, cell_ids):
    """Prism-local node indices [nc, 3 tets, 4] of the three tetrahedra of each prism (base
    cell index = cell_id // L), from the global order of the base triangle's vertices."""
    tri = mesh.cells.astype(np.int64)[np.asarray(cell_ids) // mesh.n_layers]
    p = np.argsort(tri, axis=1, kind="stable")                  # local corners by global id
    p0, p1, p2 = p[:, 0], p[:, 1], p[:, 2]
    return np.stack([np.stack([p0, p1, p2, p0 + 3], axis=1),
                     np.stack([p1, p2, p0 + 3, p1 + 3], axis=1),
                     np.stack([p2, p0 + 3, p1 + 3, p2 + 3], axis=1)], axis=1)


def _tet_geometry(X, tets):
    """Per prism and tetrahedron: basis gradients of the 6 prism nodes (zero for nodes not in
    the tetrahedron) [nc, 3, 6, 3], volumes [nc, 3] and the node weights int phi_a / V
    (1/4 on its nodes) [nc, 3, 6]."""
    nc = X.shape[0]
    Xl = _local(X)
    gradN = np.zeros((nc, 3, 6, 3))
    Nw = np.zeros((nc, 3, 6))
    vol = np.zeros((nc, 3))
    rows = np.arange(nc)
    for q in range(3):
        T = tets[:, q, :]                                         # [nc, 4]
        X0 = Xl[rows, T[:, 0]]
        M = np.stack([Xl[rows, T[:, j]] - X0 for j in (1, 2, 3)], axis=1)   # rows: edge vectors
        det = np.linalg.det(M)
        if np.any(np.abs(det) <= 0):
            raise ValueError("degenerate tetrahedron")
        G = np.linalg.inv(M)                                      # column j: gradient of phi_(j+1)
        g = np.stack([-(G[:, :, 0] + G[:, :, 1] + G[:, :, 2]), G[:, :, 0], G[:, :, 1], G[:, :, 2]], axis=1)
        for a in range(4):
            gradN[rows, q, T[:, a], :] = g[:, a, :]
            Nw[rows, q, T[:, a]] = 0.25
        vol[:, q] = np.abs(det) / 6.0
    return gradN, vol, Nw


def element_arrays(mesh, cell_ids: np.ndarray, U: np.ndarray, ref: RefElement | None = None,
                   want_jac: bool = True, picard: bool = False, xyz=None, hooks=None,
                   s_drive=None, absolute: bool = False):
    """Element residuals [nc, npe, 2] and (optionally) element Jacobians
    [nc, npe, 2, npe, 2] for the given cells.

    U may be complex (complex-step differentiation of the residual).  s_drive is a
    test-only override of the per-vertex surface used in the driving-stress term
    (the geometry always comes from the mesh's own s and H).  absolute=True returns,
    instead of the sums, the sums of the absolute values of every quadrature-point
    term (the scale of the rounding error of any summation order)."""
    ab = np.abs if absolute else (lambda x: x)
    tet = mesh.elem == "tet"
    ref = ref or RefElement("wedge" if tet else mesh.elem)
    xyz = node_xyz(mesh) if xyz is None else xyz
    nodes = cell_nodes(mesh)[cell_ids]
    X = xyz[nodes]
    Ue = U.reshape(-1, 2)[nodes]
    s_vert = mesh.surface if s_drive is None else s_drive
    s_nodes = node_column_field(mesh, s_vert)[nodes]
    if tet:     # three constant-gradient "points" per prism: its tetrahedra, weight = volume
        gradN, W, Nq = _tet_geometry(X, tet_split(mesh, cell_ids))
    else:
        gradN, W, det = _geometry(ref, X)
        if np.any(det <= 0):
            raise ValueError("non-positive Jacobian determinant")
        Nq = np.broadcast_to(ref.N, (X.shape[0],) + ref.N.shape)
    exx, eyy, exy, exz, eyz = _strain(gradN, Ue)
    q = effective_strain_rate_sq(exx, eyy, exy, exz, eyz)
    mu, dmu = viscosity(q, mesh.A, mesh.n, mesh.eps0)
    # strain-rate vectors of eq. (FOStokes)
    eps1 = np.stack([2 * exx + eyy, exy, exz], axis=-1)      # [nc, nq, 3]
    eps2 = np.stack([exy, exx + 2 * eyy, eyz], axis=-1)
    g = np.stack([np.einsum("cqi,cqai->cqa", eps1, gradN),
                  np.einsum("cqi,cqai->cqa", eps2, gradN)], axis=-1)  # [nc, nq, npe, 2]
    rg = mesh.rho * mesh.g
    sx = np.einsum("ca,cqa->cq", s_nodes, gradN[..., 0])
    sy = np.einsum("ca,cqa->cq", s_nodes, gradN[..., 1])
    grav = np.stack([sx, sy], axis=-1)                       # [nc, nq, 2]
    Re = (np.einsum("eqak->eak", ab(np.einsum("eq,eqak->eqak", W * 2 * mu, g)))
          + rg * np.einsum("eqak->eak", ab(np.einsum("eq,eqa,eqk->eqak", W, Nq, grav))))
    Je = None
    if want_jac:
        gx, gy, gz = gradN[..., 0], gradN[..., 1], gradN[..., 2]
        # derivative of eps_c . grad phi_a with respect to the (b, d) velocity dof
        Kuu = (2 * np.einsum("eqa,eqb->eqab", gx, gx) + 0.5 * np.einsum("eqa,eqb->eqab", gy, gy)
               + 0.5 * np.einsum("eqa,eqb->eqab", gz, gz))
        Kuv = np.einsum("eqa,eqb->eqab", gx, gy) + 0.5 * np.einsum("eqa,eqb->eqab", gy, gx)
        Kvu = np.einsum("eqa,eqb->eqab", gy, gx) + 0.5 * np.einsum("eqa,eqb->eqab", gx, gy)
        Kvv = (0.5 * np.einsum("eqa,eqb->eqab", gx, gx) + 2 * np.einsum("eqa,eqb->eqab", gy, gy)
               + 0.5 * np.einsum("eqa,eqb->eqab", gz, gz))
        # K[e, q, a, k, b, l]: row dof (a, k), column dof (b, l)
        K = np.stack([np.stack([Kuu, Kuv], axis=-1), np.stack([Kvu, Kvv], axis=-1)], axis=-2)
        K = K.transpose(0, 1, 2, 4, 3, 5)
        if absolute:
            Je = np.einsum("eq,eqakbl->eakbl", np.abs(W * 2 * mu), np.abs(K))
            if not picard:
                Je = Je + np.einsum("eq,eqak,eqbl->eakbl", np.abs(W * 2 * dmu), np.abs(g), np.abs(g))
        else:
            Je = np.einsum("eq,eqakbl->eakbl", W * 2 * mu, K)
            if not picard:
                Je = Je + np.einsum("eq,eqak,eqbl->eakbl", W * 2 * dmu, g, g)
    # bed friction on the lower face of the bottom layer
    L = mesh.n_layers
    bottom = (cell_ids % L) == 0
    if np.any(bottom):
        bidx = np.nonzero(bottom)[0]
        Xb = _local(X[bidx])
        tx = np.einsum("cai,ra->cri", Xb, ref.dNb[..., 0])
        ty = np.einsum("cai,ra->cri", Xb, ref.dNb[..., 1])
        dA = ref.bw[None, :] * np.linalg.norm(np.cross(tx, ty), axis=-1)   # [nb, nqb]
        beta_nodes = node_column_field(mesh, mesh.beta)[nodes[bidx]]
        beta_r = np.einsum("ca,ra->cr", beta_nodes, ref.Nb)
        ur = np.einsum("eak,ra->erk", Ue[bidx], ref.Nb)
        Re[bidx] += np.einsum("erak->eak", ab(np.einsum("er,erk,ra->erak", dA * beta_r, ur, ref.Nb)))
        if want_jac:
            M = np.einsum("erab->eab", ab(np.einsum("er,ra,rb->erab", dA * beta_r, ref.Nb, ref.Nb)))
            Je[bidx, :, 0, :, 0] += M
            Je[bidx, :, 1, :, 1] += M
    if hooks is not None:
        hooks(mesh, ref, cell_ids, nodes, X, Ue, gradN, W, Re, Je)
    return Re, Je, nodes


# --------------------------------------------------------------------------------------
# ocean back-pressure on the marine margin (Sec. 2, lateral boundary condition)
# --------------------------------------------------------------------------------------

def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def front_faces(mesh):
    """Lateral faces under ocean back-pressure: for each marked edge (a, b) of the base
    mesh (oriented so that its cell is on the left, i.e. counter-clockwise in that cell) and
    each layer k, the face with corners (a,k), (b,k), (b,k+1), (a,k+1).  Returns
    (nodes [F, 4], outward unit normal [F, 2], edge length [F], z at the corners [F, 4],
    surface s at a and b [F, 2])."""
    E = np.asarray(mesh.front_edges, dtype=np.int64).reshape(-1, 2)
    cells = mesh.cells.astype(np.int64)
    ccw = set()
    for c in cells:
        for i in range(c.shape[0]):
            ccw.add((int(c[i]), int(c[(i + 1) % c.shape[0]])))
    E = E.copy()
    for i, (a, b) in enumerate(E):
        if (a, b) in ccw and (b, a) in ccw:
            raise ValueError(f"front edge {a}-{b} is shared by two cells")
        if (b, a) in ccw and (a, b) not in ccw:
            E[i] = (b, a)
        elif (a, b) not in ccw:
            raise ValueError(f"front edge {a}-{b} is not an edge of the base mesh")
    L = mesh.n_layers
    L1 = L + 1
    d = mesh.xy[E[:, 1]] - mesh.xy[E[:, 0]]
    length = np.hypot(d[:, 0], d[:, 1])
    normal = np.stack([d[:, 1], -d[:, 0]], axis=1) / length[:, None]   # domain on the left of a -> b
    bed = mesh.surface - mesh.thickness
    z = bed[:, None] + mesh.sigma[None, :] * mesh.thickness[:, None]   # [V, L+1]
    k = np.arange(L)
    a, b = E[:, 0][:, None], E[:, 1][:, None]
    nodes = np.stack([a * L1 + k, b * L1 + k, b * L1 + k + 1, a * L1 + k + 1], axis=-1).reshape(-1, 4)
    zc = np.stack([z[E[:, 0]][:, :-1], z[E[:, 1]][:, :-1], z[E[:, 1]][:, 1:], z[E[:, 0]][:, 1:]],
                  axis=-1).reshape(-1, 4)
    rep = lambda x: np.repeat(x, L, axis=0)
    sab = np.stack([mesh.surface[E[:, 0]], mesh.surface[E[:, 1]]], axis=1)
    return nodes, rep(normal), rep(length), zc, rep(sab)


def _rational_integral(T, zl, dz, t0, t1):
    """int_{t0}^{t1} T(t) zl(t)^3 / dz(t) dt for polynomials T (numpy.poly1d), zl, dz (dz linear
    and positive on [t0, t1]).  With e the slope of dz and d its smaller end value: if
    |e| <= d / 2 the pole -dz(0)/e lies at least two interval lengths away and 16-point Gauss
    is exact to rounding; otherwise N = T zl^3 is divided by (t - t_p) (t_p the pole):
    int N / dz = int S / e + N(t_p) / e * ln((t1 - t_p) / (t0 - t_p))."""
    e = dz.c[0] if dz.order == 1 else 0.0
    d = min(dz(t0), dz(t1))
    N = T * zl ** 3
    if abs(e) * (t1 - t0) <= 0.5 * d:
        x, w = _gauss(16)
        t = t0 + (t1 - t0) * x
        return float(np.sum((t1 - t0) * w * N(t) / dz(t)))
    tp = -dz.c[-1] / e
    S, rem = np.polydiv(N.c, np.array([1.0, -tp]))
    Si = np.polyint(np.poly1d(S))
    return float((Si(t1) - Si(t0)) / e + rem[-1] / e * np.log((t1 - tp) / (t0 - tp)))


def front_face_terms(mesh):
    """Nodal loads of every front face, [F, 4 nodes, 2 components]: -int phi_node p n_c dA with
    p = rho g (s - z) - rho_w g max(-z, 0).  The face lies in the vertical plane of its edge,
    parametrised by t in [0,1] along the edge and zeta in [0,1] between its two levels
    (z = zl(t) + zeta dz(t), zl and dz = zh - zl linear in t, dA = |edge| dz dt dzeta, phi
    bilinear: (1-t)(1-zeta), t(1-zeta), t zeta, (1-t) zeta for the corners (a,k), (b,k),
    (b,k+1), (a,k+1)).
    * Ice term rho g (s - z): a polynomial of degree 3 in t and 2 in zeta, integrated exactly
      by 2 x 2 Gauss.
    * Water term rho_w g z (z < 0): split in t where the sea level crosses the lower or upper
      edge of the face.  Where the whole layer is submerged the zeta integral is
      int_0^1 z Z dz dzeta = dz (zl/2 + dz/6) (Z = 1 - zeta) or dz (zl/2 + dz/3) (Z = zeta),
      a cubic in t after the T factor (2-point Gauss, exact).  Where it crosses,
      u = zeta dz from 0 to -zl gives int z Z du = -zl^2/2 - zl^3/(6 dz) (Z = 1 - zeta) or
      zl^3/(6 dz) (Z = zeta): the zl^2 part is a cubic in t (2-point Gauss), the zl^3/dz part
      is integrated by _rational_integral.
    Also returns per node |ice term| + |water term| (the scale of these entries' rounding)."""
    nodes, normal, length, zc, sab = front_faces(mesh)
    F = nodes.shape[0]
    rg, rwg = mesh.rho * mesh.g, mesh.rho_w * mesh.g
    x2, w2 = _gauss(2)
    P = np.poly1d
    Tf = [P([-1.0, 1.0]), P([1.0, 0.0])]           # 1 - t, t  (corner a, corner b)
    corner = [(0, 0), (1, 0), (1, 1), (0, 1)]      # (T index, Z index) of the face corners
    ice = np.zeros((F, 4))
    wat = np.zeros((F, 4))
    for f in range(F):
        zl0, zl1, zh1, zh0 = zc[f]
        zl = P([zl1 - zl0, zl0])
        zh = P([zh1 - zh0, zh0])
        dz = zh - zl
        sf = P([sab[f, 1] - sab[f, 0], sab[f, 0]])
        # ice term, exact 2 x 2 Gauss
        for gt in range(2):
            t = x2[gt]
            for gz in range(2):
                zeta = x2[gz]
                zz = zl(t) + zeta * dz(t)
                val = w2[gt] * w2[gz] * dz(t) * rg * (sf(t) - zz)
                for c, (ti, zi) in enumerate(corner):
                    ice[f, c] += val * (t if ti else 1 - t) * (zeta if zi else 1 - zeta)
        # water term
        br = [0.0, 1.0]
        for q in (zl, zh):
            if q.c[0] != 0:
                r = -q.c[-1] / q.c[0]
                if 0 < r < 1:
                    br.append(r)
        br = sorted(br)
        for t0, t1 in zip(br[:-1], br[1:]):
            if t1 <= t0:
                continue
            tm = 0.5 * (t0 + t1)
            if zl(tm) >= 0:
                continue                                   # dry
            full = zh(tm) <= 0
            for c, (ti, zi) in enumerate(corner):
                T = Tf[ti]
                if full:
                    g = dz * (0.5 * zl + (dz / 3.0 if zi else dz / 6.0))
                    val = sum((t1 - t0) * w2[k] * (T * g)((t0 + (t1 - t0) * x2[k])) for k in range(2))
                else:
                    sq = sum((t1 - t0) * w2[k] * (T * zl ** 2)((t0 + (t1 - t0) * x2[k])) for k in range(2))
                    cu = _rational_integral(T, zl, dz, t0, t1) / 6.0
                    val = cu if zi else -0.5 * sq - cu
                wat[f, c] += rwg * val
    ice *= length[:, None]
    wat *= length[:, None]
    tot = -(ice + wat)[:, :, None] * normal[:, None, :]
    tot_abs = (np.abs(ice) + np.abs(wat))[:, :, None] * np.abs(normal)[:, None, :]
    return nodes, tot, tot_abs


def front_load(mesh, absolute: bool = False):
    """Residual contribution [n_dofs] of the ocean fronts (zero without fronts); it does not
    depend on U.  absolute=True: the per-term scale (sum of |quadrature terms|)."""
    R = np.zeros(mesh.n_dofs)
    fe = getattr(mesh, "front_edges", None)
    if fe is None or len(fe) == 0:
        return R
    nodes, tot, tot_abs = front_face_terms(mesh)
    vals = tot_abs if absolute else tot
    dofs = 2 * nodes[:, :, None] + np.arange(2)[None, None, :]
    return R + np.bincount(dofs.ravel(), weights=vals.ravel(), minlength=mesh.n_dofs)


def _has_front(mesh):
    fe = getattr(mesh, "front_edges", None)
    return fe is not None and len(fe) > 0


def _chunks(n, size):
    for s in range(0, n, size):
        yield np.arange(s, min(n, s + size))


def assemble(mesh, U: np.ndarray, want_jac: bool = True, picard: bool = False,
             chunk: int = 20000, cells=None, hooks=None, s_drive=None):
    """Global residual R [n_dofs] and Jacobian (scipy CSR, summed duplicates)."""
    ref = RefElement("wedge" if mesh.elem == "tet" else mesh.elem)
    xyz = node_xyz(mesh)
    nd = mesh.n_dofs
    cplx = np.iscomplexobj(U)
    R = np.zeros(nd, dtype=complex if cplx else float)
    J = None
    parts = []    # per chunk, the summed element entries (explicit zeros kept: the pattern is
                  # every node pair of a cell, also pairs of a prism that share no tetrahedron)
    all_cells = np.arange(mesh.n_cells) if cells is None else np.asarray(cells)
    for ch in _chunks(all_cells.shape[0], chunk):
        ids = all_cells[ch]
        Re, Je, nodes = element_arrays(mesh, ids, U, ref, want_jac and not cplx, picard, xyz,
                                       hooks, s_drive)
        dofs = (2 * nodes[:, :, None] + np.arange(2)[None, None, :]).reshape(ids.shape[0], -1)
        R += np.bincount(dofs.ravel(), weights=Re.real.reshape(-1), minlength=nd)
        if cplx:
            R += 1j * np.bincount(dofs.ravel(), weights=Re.imag.reshape(-1), minlength=nd)
            continue
        if want_jac:
            m = dofs.shape[1]
            rows = np.repeat(dofs, m, axis=1).ravel()
            cols = np.tile(dofs, (1, m)).ravel()
            parts.append(sp.coo_matrix((Je.reshape(-1), (rows, cols)), shape=(nd, nd)).tocsr().tocoo())
    if _has_front(mesh):      # per node, independent of U: exact on any row whose cells are all included
        R += front_load(mesh)
    if want_jac and not cplx:
        # one conversion of all chunks' entries: a sum of sparse matrices would drop the
        # structural zeros
        J = sp.coo_matrix((np.concatenate([q.data for q in parts]),
                           (np.concatenate([q.row for q in parts]), np.concatenate([q.col for q in parts]))),
                          shape=(nd, nd)).tocsr()
        J.sum_duplicates()
        J.sort_indices()
    return R, J


def residual(mesh, U, **kw):
    return assemble(mesh, U, want_jac=False, **kw)[0]


def _row_sums_and_matrix(mesh, U, picard, chunk, cells, absolute):
    """Sum over cells of |R_e,i| and the CSR matrix of sum over cells of |J_e,ij|, where
    R_e, J_e are the element arrays (absolute=False) or, per element, the sums of the
    absolute values of their quadrature-point terms (absolute=True)."""
    ref = RefElement("wedge" if mesh.elem == "tet" else mesh.elem)
    xyz = node_xyz(mesh)
    nd = mesh.n_dofs
    rs = np.zeros(nd)
    Jabs = None
    all_cells = np.arange(mesh.n_cells) if cells is None else np.asarray(cells)
    for ch in _chunks(all_cells.shape[0], chunk):
        ids = all_cells[ch]
        Re, Je, nodes = element_arrays(mesh, ids, U, ref, True, picard, xyz, absolute=absolute)
        dofs = (2 * nodes[:, :, None] + np.arange(2)[None, None, :]).reshape(ids.shape[0], -1)
        rs += np.bincount(dofs.ravel(), weights=np.abs(Re).reshape(-1), minlength=nd)
        m = dofs.shape[1]
        rows = np.repeat(dofs, m, axis=1).ravel()
        cols = np.tile(dofs, (1, m)).ravel()
        Jc = sp.coo_matrix((np.abs(Je).reshape(-1), (rows, cols)), shape=(nd, nd)).tocsr()
        Jabs = Jc if Jabs is None else Jabs + Jc
    if _has_front(mesh):
        nodes, tot, tot_abs = front_face_terms(mesh)
        dofs = 2 * nodes[:, :, None] + np.arange(2)[None, None, :]
        rs += np.bincount(dofs.ravel(), weights=(tot_abs if absolute else np.abs(tot)).ravel(), minlength=nd)
    Jabs.sum_duplicates()
    Jabs.sort_indices()
    return rs, Jabs


def abs_terms(mesh, U, picard=False, chunk=20000, cells=None):
    """Per-entry scales: S^R_i = sum over cells and quadrature points of the absolute values
    of the terms summed into R_i, and the CSR matrix S^J_ij of the same for J_ij."""
    return _row_sums_and_matrix(mesh, U, picard, chunk, cells, absolute=True)


def abs_scales(mesh, U, picard=False, chunk=20000, cells=None):
    """Row scales for rounding-level parity: S^R_i (abs_terms) and max_j S^J_ij
    (optionally from a subset of cells: exact for rows whose cells are all included).  Any
    summation order of the same terms differs from another by at most a small multiple of
    the unit roundoff times these sums."""
    rs, Jabs = abs_terms(mesh, U, picard, chunk, cells)
    jrow = np.asarray(Jabs.max(axis=1).todense()).ravel()
    return rs, jrow


def element_scales(mesh, U, picard=False, chunk=20000, cells=None):
    """Element-level row scales: sum_e |R_e,i| and max_j sum_e |J_e,ij| over the element
    residuals and Jacobians.  They lie below the per-term scales of abs_scales wherever the
    terms inside one element cancel."""
    rs, Je = _row_sums_and_matrix(mesh, U, picard, chunk, cells, absolute=False)
    return rs, np.asarray(Je.max(axis=1).todense()).ravel()


def cells_touching_nodes(mesh, nodes_sel: np.ndarray) -> np.ndarray:
    """All cells that contain at least one of the given global nodes."""
    cn = cell_nodes(mesh)
    mark = np.zeros(mesh.n_nodes, dtype=bool)
    mark[np.asarray(nodes_sel)] = True
    return np.nonzero(mark[cn].any(axis=1))[0]


def assemble_rows(mesh, U, dofs_sel: np.ndarray, picard: bool = False):
    """Residual entries and Jacobian rows (CSR restricted to the selected rows) computed
    from only the cells around the selected dofs: lets a huge mesh be spot-checked."""
    dofs_sel = np.asarray(dofs_sel, dtype=np.int64)
    cells = cells_touching_nodes(mesh, dofs_sel // 2)
    R, J = assemble(mesh, U, want_jac=True, picard=picard, cells=cells)
    return R[dofs_sel], J[dofs_sel], cells


# --------------------------------------------------------------------------------------
# energy functional (the residual is its gradient; used as a pin)
# --------------------------------------------------------------------------------------

def energy(mesh, U, s_drive=None):
    """E(U) = sum_q W [A^(-1/n) 2n/(n+1) (q+eps0^2)^((n+1)/(2n)) + rho g grad s . (u,v)]
    + 1/2 sum_bed W^b beta (u^2 + v^2)."""
    tet = mesh.elem == "tet"
    ref = RefElement("wedge" if tet else mesh.elem)
    xyz = node_xyz(mesh)
    nodes = cell_nodes(mesh)
    X = xyz[nodes]
    Ue = U.reshape(-1, 2)[nodes]
    s_nodes = node_column_field(mesh, mesh.surface if s_drive is None else s_drive)[nodes]
    if tet:
        gradN, W, Nq = _tet_geometry(X, tet_split(mesh, np.arange(mesh.n_cells)))
    else:
        gradN, W, _ = _geometry(ref, X)
        Nq = np.broadcast_to(ref.N, (X.shape[0],) + ref.N.shape)
    exx, eyy, exy, exz, eyz = _strain(gradN, Ue)
    q = effective_strain_rate_sq(exx, eyy, exy, exz, eyz)
    n = mesh.n
    dens = mesh.A ** (-1.0 / n) * (2 * n / (n + 1)) * (q + mesh.eps0 ** 2) ** ((n + 1) / (2 * n))
    uq = np.einsum("ca,cqa->cq", Ue[..., 0], Nq)
    vq = np.einsum("ca,cqa->cq", Ue[..., 1], Nq)
    sx = np.einsum("ca,cqa->cq", s_nodes, gradN[..., 0])
    sy = np.einsum("ca,cqa->cq", s_nodes, gradN[..., 1])
    E = np.sum(W * (dens + mesh.rho * mesh.g * (sx * uq + sy * vq)))
    L = mesh.n_layers
    bidx = np.arange(0, mesh.n_cells, L)
    Xb = _local(X[bidx])
    tx = np.einsum("cai,ra->cri", Xb, ref.dNb[..., 0])
    ty = np.einsum("cai,ra->cri", Xb, ref.dNb[..., 1])
    dA = ref.bw[None, :] * np.linalg.norm(np.cross(tx, ty), axis=-1)
    beta_r = np.einsum("ca,ra->cr", node_column_field(mesh, mesh.beta)[nodes[bidx]], ref.Nb)
    ub = np.einsum("ca,ra->cr", Ue[bidx, :, 0], ref.Nb)
    vb = np.einsum("ca,ra->cr", Ue[bidx, :, 1], ref.Nb)
    return E + 0.5 * np.sum(dA * beta_r * (ub ** 2 + vb ** 2))


# --------------------------------------------------------------------------------------
# sparsity pattern of the Jacobian (every node pair that shares a cell)
# --------------------------------------------------------------------------------------

def jacobian_pattern(mesh):
    """CSR (rowptr, colidx) of all dof pairs sharing a cell, columns sorted."""
    nodes = cell_nodes(mesh)
    nd = mesh.n_dofs
    dofs = (2 * nodes[:, :, None] + np.arange(2)[None, None, :]).reshape(nodes.shape[0], -1)
    m = dofs.shape[1]
    rows = np.repeat(dofs, m, axis=1).ravel()
    cols = np.tile(dofs, (1, m)).ravel()
    P = sp.coo_matrix((np.ones(rows.shape[0], dtype=np.int8), (rows, cols)), shape=(nd, nd)).tocsr()
    P.sum_duplicates()
    P.sort_indices()
    return P.indptr.astype(np.int64), P.indices.astype(np.int64)
