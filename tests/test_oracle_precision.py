"""Rounding accuracy of the FP64 oracle on the ice-sheet mesh, against a 40-digit
evaluation of the same definitions (mpmath, written out here point by point).

The ice-sheet configuration has thin (~45 m) columns 650 km from the origin.  There the
FP64 evaluation of the isoparametric map is the ill-conditioned step; these pins fix the
oracle's error on the parity scales (per-term and element-level row scales) at such rows,
for the residual (eq. residual) and for Jacobian entries (eq. linearsystem)."""
import numpy as np
import pytest

mp = pytest.importorskip("mpmath")

from fo_inputs import config1_icesheet
from oracle import fo_oracle as fo

mp.mp.dps = 40


def _mpf(x):
    return mp.mpf(float(x))


def _exact_rows(m, U, rows, jac_cols):
    """R_i for the given rows and J_ij for the (row, column) pairs, by the definition in
    40-digit arithmetic: 3D basis gradients from the inverse of the isoparametric map at
    each point of the 3-point x 2-point wedge rule, strain rates, regularised Glen
    viscosity and its derivative, gravity from the interpolated surface (no bed term:
    the rows lie above the bed)."""
    L = m.n_layers
    ref = fo.RefElement("wedge")
    cn = fo.cell_nodes(m)
    nodes_sel = np.array(sorted({r // 2 for r in rows}))
    cells = fo.cells_touching_nodes(m, nodes_sel)
    R = {r: mp.mpf(0) for r in rows}
    J = {rc: mp.mpf(0) for rc in jac_cols}
    n = _mpf(m.n)
    rg = _mpf(m.rho) * _mpf(m.g)
    pref = mp.mpf(1) / 2 * _mpf(m.A) ** (-1 / n)
    for c in cells:
        nodes = [int(x) for x in cn[c]]
        X = []
        for nd in nodes:
            v, k = nd // (L + 1), nd % (L + 1)
            H, s = _mpf(m.thickness[v]), _mpf(m.surface[v])
            X.append([_mpf(m.xy[v, 0]), _mpf(m.xy[v, 1]), (s - H) + _mpf(m.sigma[k]) * H])
        u = [_mpf(U[2 * nd]) for nd in nodes]
        w = [_mpf(U[2 * nd + 1]) for nd in nodes]
        sn = [_mpf(m.surface[nd // (L + 1)]) for nd in nodes]
        for q in range(ref.w.shape[0]):
            dN = [[_mpf(ref.dN[q, a, j]) for j in range(3)] for a in range(6)]
            Jm = mp.matrix(3, 3)
            for i in range(3):
                for j in range(3):
                    Jm[i, j] = mp.fsum(X[a][i] * dN[a][j] for a in range(6))
            det = mp.det(Jm)
            inv = Jm ** -1
            gr = [[mp.fsum(dN[a][j] * inv[j, i] for j in range(3)) for i in range(3)] for a in range(6)]
            W = _mpf(ref.w[q]) * det
            d = lambda f, i: mp.fsum(f[a] * gr[a][i] for a in range(6))
            ux, uy, uz, vx, vy, vz = d(u, 0), d(u, 1), d(u, 2), d(w, 0), d(w, 1), d(w, 2)
            exx, eyy, exy, exz, eyz = ux, vy, (uy + vx) / 2, uz / 2, vz / 2
            qe = exx ** 2 + eyy ** 2 + exx * eyy + exy ** 2 + exz ** 2 + eyz ** 2 + _mpf(m.eps0) ** 2
            mu = pref * qe ** ((1 - n) / (2 * n))
            dmu = (1 - n) / (2 * n) * mu / qe
            e = ([2 * exx + eyy, exy, exz], [exy, exx + 2 * eyy, eyz])
            sg = (d(sn, 0), d(sn, 1))
            g = [[mp.fsum(e[cc][i] * gr[a][i] for i in range(3)) for cc in range(2)] for a in range(6)]
            for a, nd in enumerate(nodes):
                for cc in range(2):
                    r = 2 * nd + cc
                    if r in R:
                        R[r] += W * 2 * mu * g[a][cc] + rg * W * _mpf(ref.N[q, a]) * sg[cc]
            for (r, col) in J:
                a = nodes.index(r // 2) if r // 2 in nodes else -1
                b = nodes.index(col // 2) if col // 2 in nodes else -1
                if a < 0 or b < 0:
                    continue
                cc, dd = r % 2, col % 2
                x, y = gr[a], gr[b]
                if (cc, dd) == (0, 0):
                    K = 2 * x[0] * y[0] + (x[1] * y[1] + x[2] * y[2]) / 2
                elif (cc, dd) == (0, 1):
                    K = x[0] * y[1] + x[1] * y[0] / 2
                elif (cc, dd) == (1, 0):
                    K = x[1] * y[0] + x[0] * y[1] / 2
                else:
                    K = (x[0] * y[0] + x[2] * y[2]) / 2 + 2 * x[1] * y[1]
                J[(r, col)] += W * (2 * mu * K + 2 * dmu * g[a][cc] * g[b][dd])
    return R, J, cells


@pytest.fixture(scope="module")
def icesheet():
    return config1_icesheet()


def _margin_rows(m):
    """Surface-level v rows of the two thinnest columns beyond 600 km from the origin and of
    two columns the full-mesh comparison singled out (thin margin columns, x = -317 km and
    +654 km)."""
    L = m.n_layers
    far = np.nonzero(np.hypot(m.xy[:, 0], m.xy[:, 1]) > 6.0e5)[0]
    thin = far[np.argsort(m.thickness[far])[:2]]
    verts = list(thin) + [90896, 112564]
    return [2 * (int(v) * (L + 1) + L) + 1 for v in verts]


def test_oracle_rounding_on_thin_far_columns(icesheet):
    m, U = icesheet
    rows = _margin_rows(m)
    Ro, Jo = fo.assemble(m, U, cells=fo.cells_touching_nodes(m, np.array([r // 2 for r in rows])))
    jac = []
    for r in rows:
        cols = Jo.indices[Jo.indptr[r]:Jo.indptr[r + 1]]
        jac += [(r, int(c)) for c in cols[:: max(1, len(cols) // 6)]]
    R, J, cells = _exact_rows(m, U, rows, jac)
    rs, js = fo.abs_scales(m, U, cells=cells)
    ers, ejs = fo.element_scales(m, U, cells=cells)
    worst = 0.0
    for r in rows:
        d = abs(Ro[r] - float(R[r]))
        worst = max(worst, d / rs[r], d / ers[r])
        assert d <= 1e-13 * rs[r] and d <= 1e-13 * ers[r], (r, d / rs[r], d / ers[r])
    for (r, c), v in J.items():
        d = abs(Jo[r, c] - float(v))
        worst = max(worst, d / js[r], d / ejs[r])
        assert d <= 1e-13 * js[r] and d <= 1e-13 * ejs[r], (r, c, d / js[r])
    print(f"\n[oracle vs 40 digits] {len(rows)} rows, {len(J)} Jacobian entries: worst {worst:.2e}")
