"""CPU reference solvers built on the FP64 oracle (TEST INFRASTRUCTURE ONLY).

* newton_solve: damped Newton, eq. (linearsystem) of arXiv:2204.04321 Sec. 3.1:
  J(U_k) delta = -F(U_k), U_{k+1} = U_k + alpha_k delta, with each linear system
  solved exactly by a sparse direct factorisation (the paper uses GMRES with
  an AMG preconditioner; a direct solve gives the reference Newton iterate).
  Readings where the paper is silent: alpha by backtracking 1, 1/2, 1/4, ...
  (at most 10 halvings) accepting ||F(U + alpha delta)|| <= (1 - 1e-4 alpha) ||F(U)||;
  convergence when ||F(U)||_2 <= tol ||F(0)||_2.
* sia_guess: the shallow-ice velocity profile used as the plain Newton initial
  guess (not in the paper; textbook formula), with the vertex surface gradient
  taken as the area-weighted mean of the adjacent base cells' gradients and
  the sliding speed rho g H |grad s| / beta capped at 1e4 m/yr.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fo_oracle import assemble, residual


def newton_solve(mesh, U0, tol=1e-8, max_newton=50, fixed=None, fixed_values=None,
                 extra=None, s_drive=None, hooks=None, picard_steps=0, verbose=False):
    """Returns (U, info).  `fixed` marks Dirichlet dofs (test use), held at
    `fixed_values`; `hooks` adds test-only source terms to element residuals."""
    U = np.array(U0, dtype=float, copy=True)
    nd = U.shape[0]
    free = np.ones(nd, dtype=bool)
    if fixed is not None:
        free[fixed] = False
        U[fixed] = fixed_values[fixed] if fixed_values is not None else U[fixed]

    def F(V):
        r = residual(mesh, V, hooks=hooks, s_drive=s_drive)
        r[~free] = 0.0
        return r

    Uz = np.zeros(nd)
    if fixed is not None:
        Uz[fixed] = U[fixed]
    f0 = np.linalg.norm(F(Uz))
    hist = []
    R = F(U)
    nr = np.linalg.norm(R)
    hist.append(nr)
    its = 0
    res_calls, jac_calls = 2, 0
    status = "maxit"
    while its < max_newton:
        if nr <= tol * f0:
            status = "converged"
            break
        _, J = assemble(mesh, U, want_jac=True, picard=its < picard_steps, hooks=hooks,
                        s_drive=s_drive)
        jac_calls += 1
        Jf = J[free][:, free].tocsc()
        d = np.zeros(nd)
        d[free] = spla.spsolve(Jf, -R[free])
        alpha = 1.0
        accepted = False
        for _ in range(11):
            Ut = U + alpha * d
            Rt = F(Ut)
            res_calls += 1
            nt = np.linalg.norm(Rt)
            if np.isfinite(nt) and nt <= (1 - 1e-4 * alpha) * nr:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            status = "linesearch"
            break
        U, R, nr = Ut, Rt, nt
        hist.append(nr)
        its += 1
        if verbose:
            print(its, alpha, nr / f0)
    if nr <= tol * f0:
        status = "converged"
    return U, dict(status=status, newton_its=its, res_hist=np.array(hist), f0=f0,
                   residual_calls=res_calls, jacobian_calls=jac_calls)


def vertex_surface_gradient(mesh):
    """Area-weighted mean over the base cells around each vertex of the cell gradient
    of the interpolated surface (triangles: P1 gradient; quads: bilinear gradient at
    the cell centre)."""
    xy = mesh.xy
    s = mesh.surface
    c = mesh.cells.astype(np.int64)
    V = mesh.n_verts
    p = xy[c]
    if c.shape[1] == 3:
        x0, x1, x2 = p[:, 0], p[:, 1], p[:, 2]
        area2 = (x1[:, 0] - x0[:, 0]) * (x2[:, 1] - x0[:, 1]) - (x2[:, 0] - x0[:, 0]) * (x1[:, 1] - x0[:, 1])
        s0, s1, s2 = s[c[:, 0]], s[c[:, 1]], s[c[:, 2]]
        # solve [x1-x0; x2-x0] g = [s1-s0; s2-s0]
        gx = ((s1 - s0) * (x2[:, 1] - x0[:, 1]) - (s2 - s0) * (x1[:, 1] - x0[:, 1])) / area2
        gy = ((s2 - s0) * (x1[:, 0] - x0[:, 0]) - (s1 - s0) * (x2[:, 0] - x0[:, 0])) / area2
        area = 0.5 * area2
    else:
        # bilinear map at the cell centre xi = eta = 1/2
        dphi = np.array([[-0.5, -0.5], [0.5, -0.5], [0.5, 0.5], [-0.5, 0.5]])
        Jm = np.einsum("cai,aj->cij", p, dphi)               # dx_i / dxi_j
        ds = np.einsum("ca,aj->cj", s[c], dphi)              # ds / dxi_j
        det = Jm[:, 0, 0] * Jm[:, 1, 1] - Jm[:, 0, 1] * Jm[:, 1, 0]
        # grad s = J^{-T} ds/dxi
        gx = (Jm[:, 1, 1] * ds[:, 0] - Jm[:, 1, 0] * ds[:, 1]) / det
        gy = (-Jm[:, 0, 1] * ds[:, 0] + Jm[:, 0, 0] * ds[:, 1]) / det
        # cell area by the shoelace formula
        xs, ys = p[:, :, 0], p[:, :, 1]
        area = 0.5 * np.abs(np.sum(xs * np.roll(ys, -1, axis=1) - np.roll(xs, -1, axis=1) * ys, axis=1))
    w = np.zeros(V)
    Gx = np.zeros(V)
    Gy = np.zeros(V)
    for j in range(c.shape[1]):
        np.add.at(w, c[:, j], area)
        np.add.at(Gx, c[:, j], area * gx)
        np.add.at(Gy, c[:, j], area * gy)
    return Gx / w, Gy / w


def sia_guess(mesh, ub_cap=1e4):
    """u(z) = u_b - 2A/(n+1) (rho g)^n |grad s|^(n-1) grad s [H^(n+1) - (s-z)^(n+1)],
    u_b = -rho g H grad s / beta (speed capped at ub_cap), s - z = H (1 - sigma_k)."""
    gx, gy = vertex_surface_gradient(mesh)
    rg = mesh.rho * mesh.g
    n = mesh.n
    H = mesh.thickness
    gm = np.hypot(gx, gy)
    drive = rg * H * gm                                    # basal shear stress magnitude
    beta = mesh.beta
    capped = beta * ub_cap <= drive
    ub_speed = np.where(capped, ub_cap, drive / np.where(capped, 1.0, beta))
    with np.errstate(invalid="ignore", divide="ignore"):
        ux_dir = np.where(gm > 0, -gx / np.where(gm > 0, gm, 1.0), 0.0)
        uy_dir = np.where(gm > 0, -gy / np.where(gm > 0, gm, 1.0), 0.0)
    ubx = ub_speed * ux_dir
    uby = ub_speed * uy_dir
    coef = 2.0 * mesh.A / (n + 1) * rg ** n * gm ** (n - 1)      # [V]
    depth = H[:, None] * (1.0 - mesh.sigma[None, :])           # s - z
    shape = H[:, None] ** (n + 1) - depth ** (n + 1)           # [V, L+1]
    u = ubx[:, None] - coef[:, None] * gx[:, None] * shape
    v = uby[:, None] - coef[:, None] * gy[:, None] * shape
    return np.stack([u, v], axis=-1).reshape(-1)
