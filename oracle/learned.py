"""FP64 reference for the learned Newton initial guess (TEST INFRASTRUCTURE ONLY).

Not in the paper: a small per-column network predicts the initial velocity profile
of each vertex column from column features; the Newton solve of Sec. 3.1 (eq.
linearsystem) then starts from it.  The method it serves is assessed only by the
Newton outcome (the network is not unique).  Definitions used by both this
reference and the GPU kernels:

* features of vertex column v (10 values): H, ds/dx, ds/dy (area-weighted mean of
  the adjacent base cells' gradients, as for the shallow-ice guess), log(max(beta,
  1e-3)), and the thickness of 6 neighbouring columns: the base-mesh neighbours of
  v, the 6 nearest kept when there are more (distance, then index), ordered by
  angle measured counter-clockwise from the downslope direction -grad s (from the
  +x axis when grad s = 0), ties by index; repeated H_v pads to 6;
* network: 10 -> 128 -> 128 -> 128 -> 22, tanh on hidden layers, linear output;
  BF16 (round to nearest even) copies of inputs, weights and hidden activations
  feed every product, sums are accumulated in FP32 on the GPU (FP64 here), biases
  and the tanh derivative use the unrounded FP32 activations;
* outputs: asinh((u - u_sia) / 10 m/yr) for (u, v) at the L+1 levels, in dof order: the
  network corrects the shallow-ice profile (which carries the rate factor A and the
  surface slope), so U = U_sia + 10 sinh(y);
* feature normalisation: column means and standard deviations (n - 1 denominator)
  plus 1e-6 over the training features;
* the guess: U = U_sia + D with D = 10 sinh(y), after k Jacobi sweeps over the base
  mesh D_v <- (D_v + mean of D_w over the base neighbours w of v) / 2, each dof of a
  column separately;
* loss: mean squared error over the batch and the 22 outputs;
* optimiser: Adam with bias correction.
"""
from __future__ import annotations

import numpy as np

from .solve import vertex_surface_gradient

LAYERS = (10, 128, 128, 128, 22)
OUT_SCALE = 10.0


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), via float32; returns float64 values."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def base_neighbours(mesh):
    """Sorted list of the vertices sharing a base cell with each vertex (self excluded)."""
    V = mesh.n_verts
    c = mesh.cells.astype(np.int64)
    nv = c.shape[1]
    a = np.repeat(c, nv, axis=1).ravel()
    b = np.tile(c, (1, nv)).ravel()
    keep = a != b
    key = np.unique(a[keep] * V + b[keep])
    src, dst = key // V, key % V
    ptr = np.zeros(V + 1, dtype=np.int64)
    np.add.at(ptr, src + 1, 1)
    return np.cumsum(ptr), dst


def column_features(mesh):
    V = mesh.n_verts
    gx, gy = vertex_surface_gradient(mesh)
    H = mesh.thickness
    F = np.zeros((V, 10))
    F[:, 0] = H
    F[:, 1] = gx
    F[:, 2] = gy
    F[:, 3] = np.log(np.maximum(mesh.beta, 1e-3))
    ptr, nb = base_neighbours(mesh)
    xy = mesh.xy
    for v in range(V):
        w = nb[ptr[v]:ptr[v + 1]]
        d = xy[w] - xy[v]
        if w.shape[0] > 6:
            d2 = d[:, 0] ** 2 + d[:, 1] ** 2
            order = np.lexsort((w, d2))[:6]
            w, d = w[order], d[order]
        ref = np.arctan2(-gy[v], -gx[v]) if (gx[v] != 0.0 or gy[v] != 0.0) else 0.0
        ang = np.mod(np.arctan2(d[:, 1], d[:, 0]) - ref, 2 * np.pi)
        order = np.lexsort((w, ang))
        hs = list(H[w[order]]) + [H[v]] * (6 - w.shape[0])
        F[v, 4:] = hs
    return F


def column_targets(mesh, U, U_sia):
    """asinh((U - U_sia) / 10) arranged per vertex column: [V, 2 (L+1)] in dof order."""
    return np.arcsinh((U - U_sia).reshape(mesh.n_verts, -1) / OUT_SCALE)


def targets_to_velocity(Y, U_sia):
    return U_sia + OUT_SCALE * np.sinh(Y).reshape(-1)


def feature_norm(X):
    """Means, then standard deviations (n - 1 denominator) + 1e-6, of features X [n, 10]."""
    X = np.asarray(X, dtype=np.float64)
    return np.concatenate([X.mean(axis=0), X.std(axis=0, ddof=1) + 1e-6])


def smooth_columns(mesh, D, sweeps):
    """k Jacobi sweeps of D [V, m] over the base mesh, written as loops over the neighbour
    lists: each sweep replaces D_v by the average of D_v and the mean of its neighbours."""
    ptr, nb = base_neighbours(mesh)
    D = np.array(D, dtype=np.float64, copy=True)
    for _ in range(sweeps):
        new = D.copy()
        for v in range(mesh.n_verts):
            w = nb[ptr[v]:ptr[v + 1]]
            if w.shape[0]:
                new[v] = 0.5 * (D[v] + D[w].mean(axis=0))
        D = new
    return D


def learned_velocity(mesh, Y, U_sia, sweeps=0):
    """The learned guess before its fallback check: U_sia + smoothed 10 sinh(Y)."""
    D = OUT_SCALE * np.sinh(np.asarray(Y, dtype=np.float64)).reshape(mesh.n_verts, -1)
    return U_sia + smooth_columns(mesh, D, sweeps).reshape(-1)


def init_params(rng, layers=LAYERS):
    """Glorot-uniform weights [out, in] and zero biases, as float32 values."""
    params = []
    for fan_in, fan_out in zip(layers[:-1], layers[1:]):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        W = rng.uniform(-lim, lim, (fan_out, fan_in)).astype(np.float32).astype(np.float64)
        params.append((W, np.zeros(fan_out)))
    return params


def mlp_forward(params, X, rounding=True):
    rnd = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    acts = [np.asarray(X, dtype=np.float64)]
    A = rnd(acts[0])
    n = len(params)
    Y = None
    for l, (W, b) in enumerate(params):
        Z = A @ rnd(W).T + b
        if l < n - 1:
            Af = np.tanh(Z)
            acts.append(Af)
            A = rnd(Af)
        else:
            Y = Z
    return Y, acts


def mlp_backward(params, acts, dY, rounding=True):
    """Gradients (dW_l, db_l) of a loss with dL/dY = dY."""
    rnd = bf16_round if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    grads = [None] * len(params)
    dZ = np.asarray(dY, dtype=np.float64)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        dZb = rnd(dZ)
        grads[l] = (dZb.T @ rnd(acts[l]), dZ.sum(axis=0))
        if l > 0:
            dA = dZb @ rnd(W)
            dZ = dA * (1.0 - acts[l] ** 2)
    return grads


def mse(Y, T):
    d = Y - T
    return np.mean(d * d), 2.0 * d / d.size


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
