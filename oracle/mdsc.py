"""Two-level column semicoarsening preconditioner for the Newton systems (TEST INFRASTRUCTURE
ONLY: only the tests may import this module; the product library never does).

The paper's solver (arXiv:2204.04321 Sec. 3.3) preconditions GMRES with a multigrid
hierarchy that first coarsens the extruded mesh vertically, with a matrix-dependent
prolongator built line by line from each vertical line's block-tridiagonal system solved
by LU without pivoting (Sec. 4.4), down to a single layer, and then runs aggregation AMG on
the resulting plane problem, with Chebyshev smoothing on GPUs (Sec. 4.4).  This module
writes out the preconditioner the library implements in that spirit, step by step:

  * column smoother B: block LU without pivoting of each vertex column's block-tridiagonal
    matrix (2x2 blocks per level, FP64 recursion), the stored factors rounded to FP32, the
    substitutions in FP64 (the column block preconditioner of the plain GMRES path); J P0 and
    the weights that restrict and prolong are stored in FP32 as well (any stored precision
    leaves the preconditioner a fixed linear operator, which is all right preconditioning
    needs), the plane operators are formed in FP64;
  * vertical collapse P0 (one step to a single layer): per column v and component c the
    weight vector w = B_v^{-1} e_c, e_c holding 1 at component c of every level, scaled so
    that the mean of its component-c entries is 1 (reading: the vertical profile the
    column's own operator gives a uniform load; its mean is positive for a positive definite
    column block, and a column where it is not positive or not finite falls back to e_c);
  * plane operator A1 = P0^T J P0 (2 dofs per base vertex) and the product J P0;
  * aggregation of the plane graph (vertices coupled when they share a base cell), repeated
    on the graph of aggregates until at most 64 vertices remain:
      pass 1, vertices in index order: an unassigned vertex whose neighbours are all
      unassigned becomes the root of a new aggregate {v} and its neighbours; an isolated
      vertex (no neighbour but itself) joins the open group of isolated vertices, a new
      group starting every 8 members;
      pass 2: each vertex still unassigned joins the aggregate of its lowest-numbered
      neighbour assigned in pass 1 (one always exists);
    unsmoothed (piecewise-constant, both components per vertex) transfers T and Galerkin
    operators T^T A T (reading: plain aggregation in place of smoothed aggregation; the
    smoothed form gave the same GMRES counts on the ice-sheet meshes);
  * smoother on each plane level: Chebyshev on D^{-1} A (D the 2x2 diagonal blocks) over
    [g / 30, g], g the Gershgorin bound max_i sum_j |(D^{-1} A)_ij| (reading: the paper names
    Chebyshev; the bound replaces a power-iteration estimate), of degree 2 on the first plane
    level and degree 1 (one damped Jacobi step) on the coarser ones, which gave the same GMRES
    counts on the ice-sheet meshes as degree 2 everywhere;
  * V-cycle: pre-smooth from zero, restrict the residual, recurse, prolong, post-smooth; the
    coarsest level solved exactly;
  * one application: y = V-cycle(P0^T r), z = P0 y + B (r - J P0 y) (coarse correction first,
    then the column smoother on what it leaves).

Dof order: node (v, k), component c at 2 (v (L + 1) + k) + c, as in the assembly oracle.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

COARSEST_MAX = 64          # plane vertices solved exactly
ISOLATED_GROUP = 8         # isolated vertices per aggregate
CHEB_DEGREES = (2, 1)     # first plane level, coarser levels
CHEB_RATIO = 30.0


# --------------------------------------------------------------------------------------
# column blocks and the column smoother
# --------------------------------------------------------------------------------------

def column_blocks(mesh, J) -> np.ndarray:
    """The diagonal blocks of J over each vertex column: [V, 2(L+1), 2(L+1)]."""
    nb = 2 * (mesh.n_layers + 1)
    V = mesh.n_verts
    C = sp.coo_matrix(J)
    keep = (C.row // nb) == (C.col // nb)
    out = np.zeros((V, nb, nb))
    np.add.at(out, (C.row[keep] // nb, C.row[keep] % nb, C.col[keep] % nb), C.data[keep])
    return out


def column_factors(blocks: np.ndarray, store=np.float32):
    """Block LU without pivoting of each column (Sec. 4.4 reading): with D_k, Lo_k, Up_k the
    diagonal, lower and upper 2x2 blocks of level k, S_0 = D_0, S_k = D_k - Lo_k S_{k-1}^{-1}
    Up_{k-1}.  Returns (Sinv, Lo, G) [V, L+1, 2, 2] with G_k = S_k^{-1} Up_k, computed in FP64
    and rounded to `store` (FP32, the stored precision of the library's factors)."""
    V, nb, _ = blocks.shape
    L1 = nb // 2
    blk = blocks.reshape(V, L1, 2, L1, 2)
    Sinv = np.zeros((V, L1, 2, 2))
    Lo = np.zeros((V, L1, 2, 2))
    G = np.zeros((V, L1, 2, 2))
    Gprev = np.zeros((V, 2, 2))
    for k in range(L1):
        Dk = blk[:, k, :, k, :].copy()
        if k > 0:
            Lo[:, k] = blk[:, k, :, k - 1, :]
            Dk -= Lo[:, k] @ Gprev
        Sinv[:, k] = np.linalg.inv(Dk)
        Up = blk[:, k, :, k + 1, :] if k + 1 < L1 else np.zeros((V, 2, 2))
        G[:, k] = Sinv[:, k] @ Up
        Gprev = G[:, k]
    rnd = lambda a: a.astype(store).astype(np.float64)
    return rnd(Sinv), rnd(Lo), rnd(G)


def column_solve(factors, r: np.ndarray) -> np.ndarray:
    """z = B^{-1} r column by column: forward w_k = S_k^{-1} (r_k - Lo_k w_{k-1}), backward
    z_k = w_k - G_k z_{k+1}."""
    Sinv, Lo, G = factors
    V, L1 = Sinv.shape[:2]
    rr = np.asarray(r, dtype=np.float64).reshape(V, L1, 2)
    w = np.zeros((V, L1, 2))
    for k in range(L1):
        y = rr[:, k].copy()
        if k > 0:
            y -= np.einsum("vij,vj->vi", Lo[:, k], w[:, k - 1])
        w[:, k] = np.einsum("vij,vj->vi", Sinv[:, k], y)
    z = w.copy()
    for k in range(L1 - 2, -1, -1):
        z[:, k] = w[:, k] - np.einsum("vij,vj->vi", G[:, k], z[:, k + 1])
    return z.reshape(-1)


# --------------------------------------------------------------------------------------
# vertical collapse
# --------------------------------------------------------------------------------------

def vertical_weights(blocks: np.ndarray) -> np.ndarray:
    """W [V, L+1, 2, 2]: W[v, k, c', c] = component c' at level k of B_v^{-1} e_c divided by
    the mean over k of its component-c entries (fallback e_c where that mean is not a
    positive finite number).  Solved by a dense FP64 solve per column."""
    V, nb, _ = blocks.shape
    L1 = nb // 2
    E = np.zeros((nb, 2))
    E[0::2, 0] = 1.0
    E[1::2, 1] = 1.0
    W = np.linalg.solve(blocks, np.broadcast_to(E, (V, nb, 2)))   # [V, nb, 2]
    W = W.reshape(V, L1, 2, 2)
    for c in range(2):
        mean = W[:, :, c, c].mean(axis=1)
        good = np.isfinite(mean) & (mean > 0)
        W[good, :, :, c] /= mean[good, None, None]
        W[~good, :, :, c] = 0.0
        W[~good, :, c, c] = 1.0
    return W


def collapse(mesh, W: np.ndarray):
    """P0 [n_dofs, 2 V] (sparse): column (v, c) holds W[v, :, :, c] on column v's dofs."""
    V, L1 = W.shape[:2]
    n = 2 * V * L1
    rows = np.repeat(np.arange(n), 2)
    cols = (2 * np.repeat(np.arange(V), 2 * L1)[:, None] + np.arange(2)[None, :]).reshape(-1)
    return sp.csr_matrix((W.reshape(-1), (rows, cols)), shape=(n, 2 * V))


# --------------------------------------------------------------------------------------
# plane aggregation
# --------------------------------------------------------------------------------------

def plane_graph(mesh):
    """Neighbour sets of the base vertices: vertices that share a base cell (and v itself)."""
    V = mesh.n_verts
    nbrs = [set([v]) for v in range(V)]
    for cell in np.asarray(mesh.cells):
        for a in cell:
            nbrs[int(a)].update(int(b) for b in cell)
    return [sorted(s) for s in nbrs]


def aggregate(nbrs):
    """Aggregates of a graph given as sorted neighbour lists (each containing the vertex
    itself): the two passes stated in the module docstring.  Returns (agg, n_agg)."""
    n = len(nbrs)
    agg = -np.ones(n, dtype=np.int64)
    n_agg = 0
    open_group, open_count = -1, 0
    for v in range(n):
        if agg[v] >= 0:
            continue
        others = [w for w in nbrs[v] if w != v]
        if not others:
            if open_group < 0 or open_count == ISOLATED_GROUP:
                open_group, open_count = n_agg, 0
                n_agg += 1
            agg[v] = open_group
            open_count += 1
            continue
        if all(agg[w] < 0 for w in others):
            agg[v] = n_agg
            for w in others:
                agg[w] = n_agg
            n_agg += 1
    after_pass1 = agg.copy()
    for v in range(n):
        if agg[v] >= 0:
            continue
        w = min(w for w in nbrs[v] if after_pass1[w] >= 0)
        agg[v] = after_pass1[w]
    return agg, n_agg


def coarse_graph(nbrs, agg, n_agg):
    out = [set([a]) for a in range(n_agg)]
    for v, lst in enumerate(nbrs):
        for w in lst:
            out[agg[v]].add(int(agg[w]))
    return [sorted(s) for s in out]


def transfer(agg, n_agg) -> sp.csr_matrix:
    """T [2 n, 2 n_agg]: both components of vertex v copied from aggregate agg[v]."""
    n = len(agg)
    rows = np.arange(2 * n)
    cols = 2 * np.repeat(agg, 2) + np.tile([0, 1], n)
    return sp.csr_matrix((np.ones(2 * n), (rows, cols)), shape=(2 * n, 2 * n_agg))


# --------------------------------------------------------------------------------------
# plane smoother and cycle
# --------------------------------------------------------------------------------------

def diag_block_inverse(A) -> sp.csr_matrix:
    n = A.shape[0] // 2
    C = sp.coo_matrix(A)
    keep = (C.row // 2) == (C.col // 2)
    D = np.zeros((n, 2, 2))
    np.add.at(D, (C.row[keep] // 2, C.row[keep] % 2, C.col[keep] % 2), C.data[keep])
    Di = np.linalg.inv(D)
    return sp.bsr_matrix((Di, np.arange(n), np.arange(n + 1)), shape=A.shape).tocsr()


def gershgorin(A, Dinv) -> float:
    """max_i sum_j |(D^{-1} A)_ij|, an upper bound of the spectral radius of D^{-1} A."""
    M = abs(Dinv @ A)
    return float(np.asarray(M.sum(axis=1)).max())


def chebyshev(A, Dinv, g, b, x, degree, ratio=CHEB_RATIO):
    """`degree` Chebyshev steps for A x = b preconditioned by D, over [g / ratio, g]
    (three-term recurrence: theta and delta the centre and half-width of the interval,
    sigma = theta / delta, rho_0 = 1 / sigma, d_0 = D^{-1} r_0 / theta,
    rho_k = 1 / (2 sigma - rho_{k-1}), d_k = rho_k rho_{k-1} d_{k-1} + 2 rho_k / delta D^{-1} r_k)."""
    lo = g / ratio
    theta, delta = 0.5 * (g + lo), 0.5 * (g - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = (Dinv @ (b - A @ x)) / theta
    x = x + d
    for _ in range(1, degree):
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (Dinv @ (b - A @ x))
        rho = rho_new
        x = x + d
    return x


class Hierarchy:
    """The preconditioner of one Jacobian J (FP64 values) on one mesh.  The parts that every
    application reads (column factors, J P0 and the weights of the restriction and
    prolongation) are stored rounded to `store` (FP32, as the library stores them; FP64 for
    the exactness pins); the plane operators are formed from the FP64 values."""

    def __init__(self, mesh, J, store=np.float32):
        J = sp.csr_matrix(J)
        self.J = J
        rnd = lambda a: a.astype(store).astype(np.float64)
        blocks = column_blocks(mesh, J)
        self.factors = column_factors(blocks, store=store)
        self.W = vertical_weights(blocks)
        self.P0 = collapse(mesh, self.W)
        JP = (J @ self.P0).tocsr()
        A = (self.P0.T @ JP).tocsr()
        self.JP = sp.csr_matrix((rnd(JP.data), JP.indices, JP.indptr), shape=JP.shape)
        self.P0s = collapse(mesh, rnd(self.W))
        nbrs = plane_graph(mesh)
        self.levels = []     # dicts: A, Dinv, g, agg, n_agg, T
        while len(nbrs) > COARSEST_MAX:
            agg, n_agg = aggregate(nbrs)
            Dinv = diag_block_inverse(A)
            T = transfer(agg, n_agg)
            self.levels.append(dict(A=A, Dinv=Dinv, g=gershgorin(A, Dinv), agg=agg, n_agg=n_agg, T=T))
            A = (T.T @ A @ T).tocsr()
            nbrs = coarse_graph(nbrs, agg, n_agg)
        self.A_coarse = A.toarray()

    def vcycle(self, b, level=0):
        if level == len(self.levels):
            return np.linalg.solve(self.A_coarse, b)
        lv = self.levels[level]
        A, Dinv, g, T = lv["A"], lv["Dinv"], lv["g"], lv["T"]
        deg = CHEB_DEGREES[0] if level == 0 else CHEB_DEGREES[1]
        x = chebyshev(A, Dinv, g, b, np.zeros_like(b), deg)
        x = x + T @ self.vcycle(T.T @ (b - A @ x), level + 1)
        return chebyshev(A, Dinv, g, b, x, deg)

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        y = self.vcycle(self.P0s.T @ r)
        return self.P0s @ y + column_solve(self.factors, r - self.JP @ y)
