"""Seeded generators of extruded ice-sheet meshes, geometry fields and velocity inputs.

Every array here is an *input*: base-mesh coordinates and connectivity, the
surface elevation s, thickness H, basal friction beta, the vertical levels
sigma and an input velocity field.  Nothing in this module evaluates the
first-order Stokes operator; the oracle and the HIP library both consume these
arrays unchanged.

Conventions shared by every consumer (they define the canonical ordering):
  * base vertex v has coordinates xy[v]; base cells are counter-clockwise;
  * the 3D node at base vertex ("column") v and level k (k = 0 at the bed,
    k = L at the surface) has index node = v * (L + 1) + k;
  * the velocity vector is interleaved, dof = 2 * node + c with c = 0 for u
    (x-velocity) and c = 1 for v (y-velocity);
  * node elevations are z = (s - H) + sigma_k * H.
Units: metres, years, pascals (A in Pa^-n yr^-1, beta in Pa yr m^-1,
velocities in m yr^-1).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

RHO_ICE = 910.0
GRAVITY = 9.81


@dataclass
class ExtrudedMesh:
    elem: str                 # "wedge" or "tet" (triangle base: a prism, or 3 tetrahedra, per
                              # layer) or "hex" (quadrilateral base)
    xy: np.ndarray            # [V, 2] float64, metres
    cells: np.ndarray         # [T, 3 or 4] int32, counter-clockwise base cells
    surface: np.ndarray       # [V] float64, upper-surface elevation s (m)
    thickness: np.ndarray     # [V] float64, ice thickness H > 0 (m)
    beta: np.ndarray          # [V] float64, basal friction coefficient >= 0 (Pa yr / m)
    sigma: np.ndarray         # [L + 1] float64, increasing from 0 (bed) to 1 (surface)
    A: float = 1e-16          # flow-law rate factor, Pa^-n yr^-1
    n: float = 3.0            # Glen exponent
    rho: float = RHO_ICE      # kg m^-3
    g: float = GRAVITY        # m s^-2
    eps0: float = 1e-10       # strain-rate regularisation, yr^-1
    name: str = ""
    meta: dict = field(default_factory=dict)
    front_edges: np.ndarray | None = None   # [n, 2] int32 base-vertex pairs of boundary edges under
                                            # ocean back-pressure (sea level at z = 0), or None
    rho_w: float = 1028.0                   # sea-water density, kg m^-3

    @property
    def n_layers(self) -> int:
        return int(self.sigma.shape[0]) - 1

    @property
    def n_verts(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_base_cells(self) -> int:
        return int(self.cells.shape[0])

    @property
    def n_nodes(self) -> int:
        return self.n_verts * (self.n_layers + 1)

    @property
    def n_dofs(self) -> int:
        return 2 * self.n_nodes

    @property
    def n_cells(self) -> int:
        return self.n_base_cells * self.n_layers

    @property
    def npe(self) -> int:
        return 8 if self.elem == "hex" else 6

    def with_fields(self, **kw) -> "ExtrudedMesh":
        return replace(self, **kw)


# --------------------------------------------------------------------------------------
# small helpers (ordering and smooth random fields)
# --------------------------------------------------------------------------------------

def _morton_key(xy: np.ndarray, bits: int = 16) -> np.ndarray:
    lo = xy.min(axis=0)
    span = np.maximum(xy.max(axis=0) - lo, 1e-30)
    q = np.clip(((xy - lo) / span * (2**bits - 1)).astype(np.int64), 0, 2**bits - 1)
    key = np.zeros(xy.shape[0], dtype=np.int64)
    for b in range(bits):
        key |= ((q[:, 0] >> b) & 1) << (2 * b)
        key |= ((q[:, 1] >> b) & 1) << (2 * b + 1)
    return key


def _spatial_order(xy: np.ndarray, cells: np.ndarray):
    """Renumber vertices along a Z-order curve and sort cells by centroid key."""
    perm = np.argsort(_morton_key(xy), kind="stable")
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.shape[0])
    xy2 = xy[perm]
    cells2 = inv[cells]
    cent = xy2[cells2].mean(axis=1)
    cperm = np.argsort(_morton_key(cent), kind="stable")
    return xy2, cells2[cperm].astype(np.int32)


def _smooth_field(rng: np.random.Generator, xy: np.ndarray, lam_min: float, lam_max: float,
                  n_modes: int = 64) -> np.ndarray:
    """Sum of random plane waves with log-uniform wavelengths, zero mean, unit variance."""
    lam = np.exp(rng.uniform(np.log(lam_min), np.log(lam_max), n_modes))
    th = rng.uniform(0.0, 2 * np.pi, n_modes)
    ph = rng.uniform(0.0, 2 * np.pi, n_modes)
    kx = 2 * np.pi / lam * np.cos(th)
    ky = 2 * np.pi / lam * np.sin(th)
    out = np.zeros(xy.shape[0])
    for i in range(n_modes):
        out += np.cos(kx[i] * xy[:, 0] + ky[i] * xy[:, 1] + ph[i])
    return out / np.sqrt(n_modes / 2.0)


def _orient_ccw(xy: np.ndarray, cells: np.ndarray) -> np.ndarray:
    p = xy[cells]
    if cells.shape[1] == 3:
        area2 = ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                 - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
        bad = area2 < 0
        cells = cells.copy()
        cells[bad] = cells[bad][:, [0, 2, 1]]
    return cells


# --------------------------------------------------------------------------------------
# base meshes
# --------------------------------------------------------------------------------------

def ellipse_mesh(n_points: int, a: float, b: float, rng: np.random.Generator):
    """Delaunay triangulation of ~n_points seeded points in the ellipse (x/a)^2+(y/b)^2<=1.

    Boundary points are equally spaced in arc length; interior points come from a
    hexagonal lattice jittered by +-0.3 spacing, thinned at random to the target count.
    Returns (xy [V,2], tris [T,3] int32 CCW) in Z-order.
    """
    from scipy.spatial import Delaunay

    area = np.pi * a * b
    perim = np.pi * (3 * (a + b) - np.sqrt((3 * a + b) * (a + 3 * b)))
    h = np.sqrt(area / (n_points * np.sqrt(3) / 2))
    nb = max(12, int(round(perim / h)))
    # lattice slightly denser than needed, then thinned
    h_lat = h * 0.98
    ny = int(np.ceil(b / (h_lat * np.sqrt(3) / 2))) + 1
    nx = int(np.ceil(a / h_lat)) + 1
    jj, ii = np.meshgrid(np.arange(-ny, ny + 1), np.arange(-nx, nx + 1), indexing="ij")
    px = ii * h_lat + (jj % 2) * h_lat / 2
    py = jj * h_lat * np.sqrt(3) / 2
    pts = np.stack([px.ravel(), py.ravel()], axis=1).astype(np.float64)
    pts += rng.uniform(-0.3 * h_lat, 0.3 * h_lat, pts.shape)
    am, bm = a - 0.6 * h, b - 0.6 * h
    inside = (pts[:, 0] / am) ** 2 + (pts[:, 1] / bm) ** 2 < 1.0
    pts = pts[inside]
    n_int = max(1, n_points - nb)
    if pts.shape[0] > n_int:
        keep = rng.choice(pts.shape[0], n_int, replace=False)
        pts = pts[np.sort(keep)]
    th = np.linspace(0.0, 2 * np.pi, 200001)
    dl = np.hypot(a * np.sin(th), b * np.cos(th))
    s = np.concatenate([[0.0], np.cumsum(0.5 * (dl[1:] + dl[:-1]) * np.diff(th))])
    targets = np.arange(nb) * (s[-1] / nb) + rng.uniform(0, s[-1] / nb)
    thb = np.interp(targets, s, th)
    bpts = np.stack([a * np.cos(thb), b * np.sin(thb)], axis=1)
    xy = np.concatenate([bpts, pts], axis=0)
    tri = Delaunay(xy).simplices.astype(np.int64)
    tri = _orient_ccw(xy, tri)
    p = xy[tri]
    area2 = ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
             - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    tri = tri[area2 > 1e-9 * h * h]
    used = np.unique(tri)
    remap = -np.ones(xy.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.shape[0])
    xy = xy[used]
    tri = remap[tri]
    return _spatial_order(xy, tri)


def structured_box(nx: int, ny: int, n_layers: int, lx: float, ly: float, elem: str = "hex",
                   diag: str = "alternate"):
    """Structured nx-by-ny cell grid on [0,lx]x[0,ly].  Vertex index = j*(nx+1)+i.

    elem="hex": one CCW quad per grid cell.  elem="wedge": each quad split into two
    CCW triangles (diagonal alternating cell by cell, or "fixed").
    Returns (xy, cells, sigma).
    """
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    cells = []
    for j in range(ny):
        for i in range(nx):
            v0 = j * (nx + 1) + i
            v1, v2, v3 = v0 + 1, v0 + nx + 2, v0 + nx + 1
            if elem == "hex":
                cells.append((v0, v1, v2, v3))
            else:
                if diag == "fixed" or (i + j) % 2 == 0:
                    cells.append((v0, v1, v2))
                    cells.append((v0, v2, v3))
                else:
                    cells.append((v0, v1, v3))
                    cells.append((v1, v2, v3))
    sigma = np.linspace(0.0, 1.0, n_layers + 1)
    return xy, np.asarray(cells, dtype=np.int32), sigma


def boundary_edges(cells: np.ndarray) -> np.ndarray:
    """Edges [n, 2] of the base mesh that belong to exactly one cell, each in its cell's
    counter-clockwise order (so the domain lies to the left of a -> b)."""
    nv = cells.shape[1]
    e = np.stack([cells, np.roll(cells, -1, axis=1)], axis=2).reshape(-1, 2).astype(np.int64)
    key = np.minimum(e[:, 0], e[:, 1]) * (cells.max() + 1) + np.maximum(e[:, 0], e[:, 1])
    _, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    return e[cnt[inv] == 1].astype(np.int32)


def floating_slab(elem: str = "hex", nx: int = 6, ny: int = 4, n_layers: int = 3, lx: float = 30e3,
                  ly: float = 20e3, H: float = 400.0, rho: float = RHO_ICE, rho_w: float = 1028.0,
                  jitter: float = 0.0, seed: int = 0):
    """Freely floating slab of uniform thickness H on [0,lx]x[0,ly] (flat surface
    s = (1 - rho/rho_w) H, base -(rho/rho_w) H below sea level, beta = 0), every lateral
    side an ocean front.  jitter > 0 moves the interior vertices by up to jitter x spacing."""
    xy, cells, sigma = structured_box(nx, ny, n_layers, lx, ly, elem=elem)
    if jitter > 0:
        rng = np.random.default_rng(seed)
        h = min(lx / nx, ly / ny)
        inner = (xy[:, 0] > 0) & (xy[:, 0] < lx) & (xy[:, 1] > 0) & (xy[:, 1] < ly)
        xy = xy.copy()
        xy[inner] += rng.uniform(-jitter * h, jitter * h, (int(inner.sum()), 2))
    V = xy.shape[0]
    Hv = np.full(V, H)
    s = (1.0 - rho / rho_w) * Hv
    return ExtrudedMesh(elem, xy, cells, s, Hv, np.zeros(V), sigma, rho=rho, name=f"floatslab_{elem}",
                        front_edges=boundary_edges(cells), rho_w=rho_w)


def marine_sheet(seed: int = 0, n_points: int = 1500, n_layers: int = 5, a: float = 80e3, b: float = 50e3,
                 rho: float = RHO_ICE, rho_w: float = 1028.0):
    """Marine ice sheet in an ellipse: bed rising inland from -700 m at the seaward end
    (x = a) to +600 m at x = -a, a dome surface whose ice goes afloat where it is thinner
    than flotation (there the base sits at -(rho/rho_w) H and beta = 0), log-normal beta
    on grounded ice, and ocean fronts on the boundary edges whose two vertices have the base
    below sea level.  Returns (mesh, U): U is the shallow-ice-shaped input plus 1% noise."""
    rng = np.random.default_rng(seed)
    xy, tri = ellipse_mesh(n_points, a, b, rng)
    x, y = xy[:, 0] / a, xy[:, 1] / b
    r2 = np.minimum(x * x + y * y, 1.0)
    bed = 600.0 - 1300.0 * (x + 1.0) / 2.0 + 60.0 * _smooth_field(rng, xy, 10e3, 40e3)
    H = np.maximum(60.0, 2200.0 * (1.0 - r2) ** 0.4 * (1.0 - 0.35 * (x + 1.0) / 2.0))
    afloat = H < -(rho_w / rho) * bed
    base = np.where(afloat, -(rho / rho_w) * H, bed)
    s = base + H
    beta = np.where(afloat, 0.0, np.exp(np.log(800.0) + 0.8 * _smooth_field(rng, xy, 10e3, 40e3)))
    edges = boundary_edges(tri)
    wet = (base[edges[:, 0]] < 0) & (base[edges[:, 1]] < 0)
    m = ExtrudedMesh("wedge", xy, tri, s, H, beta, np.linspace(0.0, 1.0, n_layers + 1), rho=rho,
                     A=1e-16, name="marine_sheet", front_edges=edges[wet], rho_w=rho_w)
    return m, shallow_ice_velocity(m, rng)


# --------------------------------------------------------------------------------------
# velocity inputs
# --------------------------------------------------------------------------------------

def smooth_velocity(mesh: ExtrudedMesh, rng: np.random.Generator, u_scale: float = 100.0,
                    noise_rel: float = 0.01) -> np.ndarray:
    """Smooth interleaved velocity input of magnitude ~u_scale plus Gaussian noise."""
    L = mesh.n_layers
    x = mesh.xy[:, 0][:, None]
    y = mesh.xy[:, 1][:, None]
    lx = max(np.ptp(mesh.xy[:, 0]), 1.0)
    ly = max(np.ptp(mesh.xy[:, 1]), 1.0)
    sg = mesh.sigma[None, :]
    u = u_scale * (0.75 + 0.25 * (1 - (1 - sg) ** 4)) * (
        1 + 0.1 * np.sin(2 * np.pi * x / lx) * np.cos(2 * np.pi * y / ly))
    v = 0.1 * u_scale * np.cos(2 * np.pi * x / lx) * np.sin(2 * np.pi * y / ly) * sg
    U = np.stack([u, v], axis=-1).reshape(-1)
    assert U.shape[0] == 2 * mesh.n_verts * (L + 1)
    if noise_rel > 0:
        U = U + rng.normal(0.0, noise_rel * u_scale, U.shape)
    return U


def dome_velocity(mesh: ExtrudedMesh, a: float, b: float, rng: np.random.Generator,
                  u_surf: float = 300.0, noise_rel: float = 0.01) -> np.ndarray:
    """Outward-flowing synthetic dome velocity with a quartic (shallow-ice-shaped)
    vertical profile plus 20% plug flow, and 1% Gaussian noise of the mean speed."""
    x = mesh.xy[:, 0] / a
    y = mesh.xy[:, 1] / b
    r2 = x * x + y * y
    vec = np.stack([x, y], axis=1) * (u_surf * r2)[:, None]
    sg = mesh.sigma
    prof = 0.2 + 0.8 * (1.0 - (1.0 - sg) ** 4)
    U = (vec[:, None, :] * prof[None, :, None]).reshape(-1)
    if noise_rel > 0:
        mean_speed = np.mean(np.abs(U))
        U = U + rng.normal(0.0, noise_rel * mean_speed, U.shape)
    return U


def _lsq_slope(xy: np.ndarray, cells: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Least-squares plane slope of the vertex field f over each vertex and its base-mesh
    neighbours (a generic fit; [V, 2])."""
    V = xy.shape[0]
    nv = cells.shape[1]
    a = np.repeat(cells, nv, axis=1).ravel().astype(np.int64)
    b = np.tile(cells, (1, nv)).ravel().astype(np.int64)
    key = np.unique(a[a != b] * V + b[a != b])
    src, dst = key // V, key % V
    dx = xy[dst] - xy[src]
    df = f[dst] - f[src]
    M = np.zeros((V, 2, 2))
    r = np.zeros((V, 2))
    np.add.at(M, src, dx[:, :, None] * dx[:, None, :])
    np.add.at(r, src, dx * df[:, None])
    return np.linalg.solve(M, r[:, :, None])[:, :, 0]


def shallow_ice_velocity(mesh: ExtrudedMesh, rng: np.random.Generator, noise_rel: float = 0.01,
                         sliding_cap: float = 1e4) -> np.ndarray:
    """Shallow-ice-shaped input velocity: the textbook column profile of lamellar flow,
    u(sigma) = u_b - 2A/(n+1) (rho g)^n |g|^(n-1) g [H^(n+1) - ((1 - sigma) H)^(n+1)],
    u_b = -rho g H g / beta (speed capped), driven by a least-squares surface slope g, plus
    Gaussian noise of noise_rel times the mean speed."""
    n, A, rg = mesh.n, mesh.A, mesh.rho * mesh.g
    g = _lsq_slope(mesh.xy, mesh.cells, mesh.surface)
    gn = np.sqrt((g * g).sum(axis=1))
    H = mesh.thickness
    sg = mesh.sigma
    shape = H[:, None] ** (n + 1) - ((1.0 - sg[None, :]) * H[:, None]) ** (n + 1)       # [V, L+1]
    coef = -2.0 * A / (n + 1) * rg ** n * gn ** (n - 1)
    with np.errstate(over="ignore", invalid="ignore"):
        ub = -rg * H[:, None] * g / np.maximum(mesh.beta, 1e-300)[:, None]
        ubn = np.sqrt((ub * ub).sum(axis=1))
        ub *= np.minimum(1.0, sliding_cap / np.maximum(ubn, 1e-300))[:, None]
    free = mesh.beta == 0          # no friction: sliding at the cap, down the surface slope
    if np.any(free):
        ub[free] = -sliding_cap * g[free] / np.maximum(gn[free], 1e-300)[:, None]
    U = ub[:, None, :] + (coef[:, None] * shape)[:, :, None] * g[:, None, :]
    U = U.reshape(-1)
    if noise_rel > 0:
        U = U + rng.normal(0.0, noise_rel * np.mean(np.abs(U)), U.shape)
    return U


# --------------------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------------------

def config0_slab(seed: int = 0):
    """20x20 km slab, 20x20 quads x 5 layers of Q1 hexes (2000 cells, 2646 nodes).

    H = 1000 + 200 sin(2 pi x/L) sin(2 pi y/L); planar bed b = -x tan(0.5 deg) so the
    mean surface slope is 0.5 deg; beta = 1000 (1 + sin sin); A = 1e-16, n = 3.
    Input velocity: smooth ~100 m/yr field plus 1% Gaussian noise.
    """
    rng = np.random.default_rng(seed)
    Lx = 20e3
    xy, cells, sigma = structured_box(20, 20, 5, Lx, Lx, elem="hex")
    x, y = xy[:, 0], xy[:, 1]
    ss = np.sin(2 * np.pi * x / Lx) * np.sin(2 * np.pi * y / Lx)
    H = 1000.0 + 200.0 * ss
    bed = -x * np.tan(np.deg2rad(0.5))
    mesh = ExtrudedMesh("hex", xy, cells, bed + H, H, 1000.0 * (1.0 + ss), sigma,
                        A=1e-16, n=3.0, eps0=1e-10, name="slab20x20x5")
    U = smooth_velocity(mesh, rng, 100.0, 0.01)
    return mesh, U


def _dome_fields(xy, a, b, rng, h_max, bed_amp, beta_mu, beta_sigma, lam_min, lam_max):
    r2 = (xy[:, 0] / a) ** 2 + (xy[:, 1] / b) ** 2
    g1 = _smooth_field(rng, xy, lam_min, lam_max)
    g2 = _smooth_field(rng, xy, lam_min, lam_max)
    g3 = _smooth_field(rng, xy, lam_min, lam_max)
    H = np.maximum(50.0, h_max * np.clip(1.0 - r2, 0.0, None) ** 0.375) * np.clip(1.0 + 0.05 * g1, 0.5, None)
    H *= min(1.0, h_max / H.max())
    bed = bed_amp * g2 / np.max(np.abs(g2))
    beta = np.exp(np.log(beta_mu) + beta_sigma * g3)
    return bed + H, H, beta


def config1_icesheet(seed: int = 1, n_points: int = 125_000, n_layers: int = 10):
    """Ice-sheet-scale wedge mesh: Delaunay of ~125k points in a 1500 x 700 km ellipse,
    extruded to 10 uniform layers (~250k triangles, ~2.5M wedges, ~2.75M dofs).

    Smooth seeded dome H (max 3000 m), smooth bed +-500 m, log-normal beta
    (mu = ln 500, sigma = 1), A = 1e-16; input velocity: the shallow-ice column profile
    plus 1% noise.
    """
    rng = np.random.default_rng(seed)
    a, b = 750e3, 350e3
    xy, tri = ellipse_mesh(n_points, a, b, rng)
    s, H, beta = _dome_fields(xy, a, b, rng, 3000.0, 500.0, 500.0, 1.0, 30e3, 200e3)
    sigma = np.linspace(0.0, 1.0, n_layers + 1)
    mesh = ExtrudedMesh("wedge", xy, tri, s, H, beta, sigma, A=1e-16, name="icesheet125k",
                        meta={"a": a, "b": b})
    U = shallow_ice_velocity(mesh, rng)
    return mesh, U


def ensemble_member(m: int, n_layers: int = 10, tri_range=(10_000, 200_000)):
    """Ensemble member m (seed 1000+m): T ~ U[10k, 200k] base triangles in the 1500 x 700 km
    ellipse, log-beta standard deviation ~ U[0.5, 1.5], A ~ U[0.5e-16, 2e-16]."""
    rng = np.random.default_rng(1000 + m)
    T = int(rng.integers(tri_range[0], tri_range[1] + 1))
    sig_b = float(rng.uniform(0.5, 1.5))
    A = float(rng.uniform(0.5e-16, 2e-16))
    a, b = 750e3, 350e3
    xy, tri = ellipse_mesh(T // 2 + 2, a, b, rng)
    s, H, beta = _dome_fields(xy, a, b, rng, 3000.0, 500.0, 500.0, sig_b, 30e3, 200e3)
    sigma = np.linspace(0.0, 1.0, n_layers + 1)
    mesh = ExtrudedMesh("wedge", xy, tri, s, H, beta, sigma, A=A, name=f"member{m}",
                        meta={"a": a, "b": b, "beta_sigma": sig_b})
    U = dome_velocity(mesh, a, b, rng)
    return mesh, U


def learned_mesh(seed: int, n_points: int = 2000, n_layers: int = 10):
    """Small ice cap for the learned initial guess (~4k triangles, ~40k wedges).

    Semi-axes a ~ U[80,150] km, aspect ~ U[0.4,0.8]; H_max ~ U[1500,3000] m; bed +-500 m;
    log-beta sigma ~ U[0.5,1.5] around ln 500; A ~ U[0.5e-16, 2e-16]."""
    rng = np.random.default_rng(seed)
    a = float(rng.uniform(80e3, 150e3))
    b = a * float(rng.uniform(0.4, 0.8))
    h_max = float(rng.uniform(1500.0, 3000.0))
    sig_b = float(rng.uniform(0.5, 1.5))
    A = float(rng.uniform(0.5e-16, 2e-16))
    xy, tri = ellipse_mesh(n_points, a, b, rng)
    s, H, beta = _dome_fields(xy, a, b, rng, h_max, 500.0, 500.0, sig_b, 20e3, 100e3)
    sigma = np.linspace(0.0, 1.0, n_layers + 1)
    return ExtrudedMesh("wedge", xy, tri, s, H, beta, sigma, A=A, name=f"cap{seed}",
                        meta={"a": a, "b": b, "h_max": h_max, "beta_sigma": sig_b})


def box_hex_single(hx: float, hy: float, hz: float, beta: float = 0.0, slope_x: float = 0.0,
                   slope_y: float = 0.0):
    """One box hexahedron [0,hx]x[0,hy]x[0,hz]; flat bed at z=0; the surface field s
    carries the given slopes (it drives gravity only; the geometry stays a box)."""
    xy = np.array([[0, 0], [hx, 0], [hx, hy], [0, hy]], dtype=np.float64)
    cells = np.array([[0, 1, 2, 3]], dtype=np.int32)
    H = np.full(4, hz)
    return ExtrudedMesh("hex", xy, cells, H.copy(), H, np.full(4, beta), np.array([0.0, 1.0]),
                        name="boxhex", meta={"slope": (slope_x, slope_y)})


def right_wedge_single(hx: float, hy: float, hz: float, beta: float = 0.0):
    """One right-angled wedge: base triangle (0,0),(hx,0),(0,hy), height hz."""
    xy = np.array([[0, 0], [hx, 0], [0, hy]], dtype=np.float64)
    cells = np.array([[0, 1, 2]], dtype=np.int32)
    H = np.full(3, hz)
    return ExtrudedMesh("wedge", xy, cells, H.copy(), H, np.full(3, beta), np.array([0.0, 1.0]),
                        name="rightwedge")


def perturbed(mesh: ExtrudedMesh, rng: np.random.Generator, rel: float = 0.2) -> ExtrudedMesh:
    """Jitter every base vertex by up to rel * (local spacing) and perturb H, s, beta
    smoothly, keeping all cells valid; returns a new mesh (for unstructured test cases)."""
    xy = mesh.xy.copy()
    span = np.ptp(xy, axis=0)
    h = np.sqrt(span[0] * span[1] / max(mesh.n_base_cells, 1))
    xy += rng.uniform(-rel * h, rel * h, xy.shape)
    H = mesh.thickness * (1.0 + 0.2 * rng.uniform(-1, 1, mesh.n_verts))
    s = mesh.surface + 0.1 * mesh.thickness * rng.uniform(-1, 1, mesh.n_verts)
    beta = mesh.beta * np.exp(0.5 * rng.normal(size=mesh.n_verts))
    return replace(mesh, xy=xy, thickness=H, surface=s, beta=beta, name=mesh.name + "_pert")
