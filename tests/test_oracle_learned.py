"""Pins of the learned-guess reference (no GPU): BF16 rounding against torch's own
conversion, MLP gradients against finite differences, Adam's first step in closed
form, and column features on hand-built meshes with known answers."""
import numpy as np
import pytest
import torch

from fo_inputs.meshgen import ExtrudedMesh
from oracle import learned as ol


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-20, 20, 10000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 65504.0, 1e-38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ol.bf16_round(x), ref)
    # ties go to even
    assert ol.bf16_round(1.0 + 2 ** -8) == 1.0
    assert ol.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def _small_params(rng, layers=(10, 7, 6, 5, 4)):
    return [(rng.normal(size=(o, i)) / np.sqrt(i), rng.normal(size=o) * 0.1)
            for i, o in zip(layers[:-1], layers[1:])]


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    params = _small_params(rng)
    X = rng.normal(size=(9, 10))
    T = rng.normal(size=(9, 4))

    def loss(ps):
        Y, _ = ol.mlp_forward(ps, X, rounding=False)
        return ol.mse(Y, T)[0]

    Y, acts = ol.mlp_forward(params, X, rounding=False)
    _, dY = ol.mse(Y, T)
    grads = ol.mlp_backward(params, acts, dY, rounding=False)
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
                old = arr[idx]
                arr[idx] = old + h
                lp = loss(params)
                arr[idx] = old - h
                lm = loss(params)
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g[idx]) <= 1e-7 * max(1.0, abs(fd)), (l, idx, fd, g[idx])


def test_bf16_gradients_close_to_exact_ones():
    rng = np.random.default_rng(2)
    params = ol.init_params(rng)
    X = rng.normal(size=(64, 10))
    T = rng.normal(size=(64, 22)) * 0.3
    Y0, a0 = ol.mlp_forward(params, X, rounding=False)
    Y1, a1 = ol.mlp_forward(params, X, rounding=True)
    assert np.linalg.norm(Y1 - Y0) <= 2e-2 * np.linalg.norm(Y0)
    g0 = ol.mlp_backward(params, a0, ol.mse(Y0, T)[1], rounding=False)
    g1 = ol.mlp_backward(params, a1, ol.mse(Y1, T)[1], rounding=True)
    for (w0, b0), (w1, b1) in zip(g0, g1):
        assert np.linalg.norm(w1 - w0) <= 5e-2 * np.linalg.norm(w0)


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    p1, m, v = ol.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), rtol=1e-14)


def _fan_mesh(angles_deg, radii, Hs, slope=(-0.01, 0.0)):
    """Centre vertex 0 with neighbours on a fan; surface s = slope . x + 1000."""
    ang = np.deg2rad(np.asarray(angles_deg))
    xy = np.concatenate([[[0.0, 0.0]], np.stack([radii * np.cos(ang), radii * np.sin(ang)], 1)])
    n = len(angles_deg)
    cells = np.array([[0, 1 + i, 1 + (i + 1) % n] for i in range(n)], dtype=np.int32)
    H = np.concatenate([[500.0], Hs])
    s = 1000.0 + slope[0] * xy[:, 0] + slope[1] * xy[:, 1]
    return ExtrudedMesh("wedge", xy, cells, s, H, np.full(n + 1, 300.0), np.linspace(0, 1, 4))


def test_features_neighbour_order_and_values():
    # six neighbours at 10, 70, ..., 310 degrees; downslope is +x for s = -0.01 x
    m = _fan_mesh([10, 70, 130, 190, 250, 310], np.full(6, 1e3), [11.0, 12, 13, 14, 15, 16])
    F = ol.column_features(m)
    np.testing.assert_allclose(F[0, 0], 500.0)
    np.testing.assert_allclose(F[0, 1:3], [-0.01, 0.0], atol=1e-15)
    np.testing.assert_allclose(F[0, 3], np.log(300.0))
    np.testing.assert_array_equal(F[0, 4:], [11.0, 12, 13, 14, 15, 16])
    # downslope towards +y (s = -0.01 y): ordering starts at the 90-degree direction
    m2 = _fan_mesh([10, 70, 130, 190, 250, 310], np.full(6, 1e3), [11.0, 12, 13, 14, 15, 16], (0.0, -0.01))
    np.testing.assert_array_equal(ol.column_features(m2)[0, 4:], [13.0, 14, 15, 16, 11, 12])


def test_features_keep_six_nearest_and_pad():
    # no neighbour exactly on the downslope ray (its side of the cut would be decided by rounding)
    ang = [10, 55, 100, 145, 190, 235, 280, 325]
    radii = np.array([1e3, 3e3, 1e3, 3e3, 1e3, 1e3, 1e3, 1e3])   # the two far ones are dropped
    m = _fan_mesh(ang, radii, np.arange(21.0, 29.0))
    F = ol.column_features(m)
    np.testing.assert_array_equal(F[0, 4:], [21.0, 23, 25, 26, 27, 28])
    # a corner vertex of the fan has 3 neighbours: padded with its own H
    assert np.sum(F[1, 4:] == m.thickness[1]) == 3


def test_target_transform_roundtrip():
    m = _fan_mesh([0, 120, 240], np.full(3, 1e3), [1.0, 2, 3])
    rng = np.random.default_rng(3)
    U = rng.normal(size=m.n_dofs) * 300
    Us = rng.normal(size=m.n_dofs) * 300
    np.testing.assert_allclose(ol.targets_to_velocity(ol.column_targets(m, U, Us), Us), U, rtol=1e-12)
    np.testing.assert_array_equal(ol.column_targets(m, Us, Us), 0.0)


def test_smoothing_pins():
    """Jacobi smoothing of the correction: a field constant over the mesh is unchanged, one
    sweep of a single spike gives the spike half its value and each neighbour the spike over
    twice its neighbour count, and many sweeps drive any field towards a constant."""
    from fo_inputs import learned_mesh
    m = learned_mesh(20002, n_points=120)
    ptr, nb = ol.base_neighbours(m)
    const = np.full((m.n_verts, 3), 4.5)
    np.testing.assert_allclose(ol.smooth_columns(m, const, 7), const, rtol=1e-15)
    D = np.zeros((m.n_verts, 1))
    D[10] = 8.0
    S = ol.smooth_columns(m, D, 1)
    assert S[10, 0] == 4.0
    for w in nb[ptr[10]:ptr[11]]:
        deg_w = ptr[w + 1] - ptr[w]
        assert abs(S[w, 0] - 0.5 * 8.0 / deg_w) <= 1e-15
    far = np.setdiff1d(np.arange(m.n_verts), np.concatenate([[10], nb[ptr[10]:ptr[11]]]))
    assert np.all(S[far, 0] == 0.0)
    R = np.random.default_rng(0).normal(size=(m.n_verts, 2))
    S = ol.smooth_columns(m, R, 400)
    assert S.std(axis=0).max() < 1e-2 * R.std(axis=0).min()


def test_feature_norm_pins():
    X = np.array([[1.0] * 10, [3.0] * 10, [5.0] * 10])
    n = ol.feature_norm(X)
    np.testing.assert_allclose(n[:10], 3.0)
    np.testing.assert_allclose(n[10:], 2.0 + 1e-6)    # sqrt((4 + 0 + 4) / 2)


def test_targets_roundtrip():
    from fo_inputs import learned_mesh
    m = learned_mesh(20003, n_points=80)
    rng = np.random.default_rng(1)
    Us = rng.normal(size=m.n_dofs) * 50
    U = Us + rng.normal(size=m.n_dofs) * 30
    Y = ol.column_targets(m, U, Us)
    np.testing.assert_allclose(ol.targets_to_velocity(Y, Us), U, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(ol.learned_velocity(m, Y, Us, 0), U, rtol=1e-12, atol=1e-9)
