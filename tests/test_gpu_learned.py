"""GPU kernels of the learned initial guess against the FP64 reference with the same BF16
rounding points: features (exact ordering), forward/backward (normwise 1e-3), MSE gradient
and Adam (FP32 rounding), and a small train-then-solve run showing the gain."""
import numpy as np
import pytest
import torch

from fo_inputs import learned_mesh
from oracle import learned as ol
from oracle import solve

from gpu_util import gpu_mesh, to_dev

pytestmark = pytest.mark.gpu


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)


def _unflat(vec):
    out, o = [], 0
    for i, j in zip(ol.LAYERS[:-1], ol.LAYERS[1:]):
        W = vec[o:o + i * j].reshape(j, i); o += i * j
        b = vec[o:o + j]; o += j
        out.append((W.astype(np.float64), b.astype(np.float64)))
    return out


def test_features_match_reference():
    m = learned_mesh(20001)
    M = gpu_mesh(m)
    F = M.features().cpu().numpy()
    Fo = ol.column_features(m)
    np.testing.assert_allclose(F[:, :4], Fo[:, :4], rtol=1e-6, atol=1e-9)
    # neighbour thicknesses are copied values: the ordering must match exactly
    np.testing.assert_array_equal(F[:, 4:], Fo[:, 4:].astype(np.float32))
    mu, sd = Fo.mean(0), Fo.std(0) + 1e-12
    norm = torch.tensor(np.concatenate([mu, sd]), dtype=torch.float32, device="cuda")
    Fn = M.features(norm).cpu().numpy()
    np.testing.assert_allclose(Fn, (Fo - mu) / sd, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("B", [1, 37, 512])
def test_forward_backward_match_reference(B):
    from paper_2204_04321_amd.api import MLP
    rng = np.random.default_rng(B)
    params = ol.init_params(rng)
    for W, b in params:
        b[:] = rng.normal(size=b.shape) * 0.1
    flat = _flat(params)
    params = _unflat(flat.astype(np.float64))
    X = rng.normal(size=(B, 10)).astype(np.float32)
    T = (rng.normal(size=(B, 22)) * 0.5).astype(np.float32)
    net = MLP(torch.from_numpy(flat).cuda())
    Xd = torch.from_numpy(X).cuda()
    Y, acts = net.forward(Xd)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    dY = MLP.mse_grad(Y, torch.from_numpy(T).cuda(), loss)
    G = net.backward(Xd, acts, dY)
    torch.cuda.synchronize()
    Yo, ao = ol.mlp_forward(params, X.astype(np.float64))
    lo, dYo = ol.mse(Yo, T.astype(np.float64))
    Go = _flat([(w, b) for w, b in ol.mlp_backward(params, ao, dYo)])
    Yg = Y.cpu().numpy()
    assert np.linalg.norm(Yg - Yo) <= 1e-3 * np.linalg.norm(Yo)
    assert abs(loss.item() - lo) <= 1e-3 * lo
    Gg = G.cpu().numpy()
    o = 0
    for i, j in zip(ol.LAYERS[:-1], ol.LAYERS[1:]):
        for size in (i * j, j):
            a, r = Gg[o:o + size], Go[o:o + size]
            assert np.linalg.norm(a - r) <= 1e-3 * np.linalg.norm(r) + 1e-12, (i, j, size)
            o += size


def test_adam_matches_reference():
    from paper_2204_04321_amd.api import MLP
    rng = np.random.default_rng(5)
    n = 37270
    p = rng.normal(size=n).astype(np.float32)
    net = MLP(torch.from_numpy(p.copy()).cuda())
    m = np.zeros(n); v = np.zeros(n); pr = p.astype(np.float64)
    for t in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        net.grads.copy_(torch.from_numpy(g))
        net.adam(lr=1e-2)
        pr, m, v = ol.adam_step(pr, g.astype(np.float64), m, v, t, lr=1e-2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(net.params.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)


def test_targets_and_feature_stats_match_reference():
    from paper_2204_04321_amd.api import MLP
    m = learned_mesh(20004, n_points=600)
    M = gpu_mesh(m)
    rng = np.random.default_rng(3)
    Us = solve.sia_guess(m)
    U = Us + rng.normal(size=m.n_dofs) * 40
    T = M.learned_targets(to_dev(U), to_dev(Us)).cpu().numpy()
    np.testing.assert_allclose(T, ol.column_targets(m, U, Us), rtol=2e-7, atol=1e-7)
    X = rng.normal(size=(5000, 10)) * np.arange(1, 11) + np.arange(10) * 100.0
    X = X.astype(np.float32)
    norm, Xn = MLP.feature_stats(torch.from_numpy(X).cuda(), normalised=True)
    ref = ol.feature_norm(X.astype(np.float64))
    np.testing.assert_allclose(norm.cpu().numpy(), ref, rtol=1e-6)
    # (x - mean) / std in FP32 from FP32-rounded statistics: besides a few ulps of the
    # result, the FP32 rounding of x and of the mean, relative to the column's spread
    exact = (X.astype(np.float64) - ref[:10]) / ref[10:]
    slack = 2.0 * (np.spacing(np.abs(X).max(0)).astype(np.float64) + np.spacing(np.abs(ref[:10]).astype(np.float32))) / ref[10:]
    assert np.all(np.abs(Xn.cpu().numpy() - exact) <= 1e-6 * np.abs(exact) + slack)


@pytest.mark.parametrize("sweeps", [0, 5])
def test_smoothed_guess_matches_reference(sweeps):
    """U = U_sia + smoothed 10 sinh(Y) (no fallback) against the reference composition, with
    the reference's own features, normalisation and BF16-rounded network."""
    m = learned_mesh(20005, n_points=500)
    M = gpu_mesh(m)
    rng = np.random.default_rng(sweeps + 11)
    params = ol.init_params(rng)
    for W, b in params:
        b[:] = rng.normal(size=b.shape) * 0.1
    flat = _flat(params)
    params = _unflat(flat.astype(np.float64))
    Fo = ol.column_features(m)
    nrm = ol.feature_norm(Fo)
    U, used = M.learned_guess(torch.from_numpy(flat).cuda(), torch.tensor(nrm, dtype=torch.float32).cuda(),
                              fallback=0, smooth=sweeps)
    assert used
    Y, _ = ol.mlp_forward(params, ((Fo - nrm[:10]) / nrm[10:]).astype(np.float32).astype(np.float64))
    Us = solve.sia_guess(m)
    Uref = ol.learned_velocity(m, Y, Us, sweeps)
    d = U.cpu().numpy() - Uref
    print(f"\n[learned guess, {sweeps} sweeps] |dU| / |D| = {np.linalg.norm(d) / np.linalg.norm(Uref - Us):.2e}")
    assert np.linalg.norm(d) <= 3e-3 * np.linalg.norm(Uref - Us)


def test_newton_learned_init_reports_the_guess():
    """FO_INIT_LEARNED inside fo_newton_solve starts from the same guess as
    fo_initial_guess_learned and reports which guess it used."""
    m = learned_mesh(20006, n_points=500)
    M = gpu_mesh(m)
    rng = np.random.default_rng(4)
    flat = torch.from_numpy(_flat(ol.init_params(rng))).cuda()
    nrm = torch.tensor(ol.feature_norm(ol.column_features(m)), dtype=torch.float32).cuda()
    for fb in (0, 1):
        U0, used = M.learned_guess(flat, nrm, fallback=fb, smooth=3)
        U = torch.zeros(M.n_dofs, dtype=torch.float64, device="cuda")
        rep = M.newton_solve(U, init="learned", mlp_params=flat, mlp_norm=nrm, learned_fallback=fb,
                             learned_smooth=3, max_newton=0)
        assert rep["status"] == -6           # the iteration cap of 0: U holds the starting guess
        assert torch.equal(U, U0)
        assert rep["learned_fallbacks"] == (0 if used else 1)
        assert rep["init_used"] == (2 if used else 1)
        rep = M.newton_solve(U, init="learned", mlp_params=flat, mlp_norm=nrm, learned_fallback=fb, learned_smooth=3)
        assert rep["status"] == 0, rep
    with pytest.raises(Exception):
        M.newton_solve(U, init="learned", check_status=True)      # no network given


def test_learned_guess_training_and_fallback():
    """Train on solutions the method generates (small meshes), then start Newton on held-out
    meshes from the learned guess and from the shallow-ice guess.  Asserted: training lowers
    the loss, every solve converges, and the residual-checked fallback keeps the network's
    guess only when its residual norm is no larger than the shallow-ice guess's (otherwise it
    returns the shallow-ice guess bit for bit).  The Newton counts of both starts are printed:
    the per-column network is not required to win on these steep synthetic caps."""
    from paper_2204_04321_amd.api import Mesh
    from paper_2204_04321_amd.learned import collect, evaluate, train
    train_set = collect(range(30000, 30040), n_points=500)
    model = train(train_set, epochs=150, batch=2048, seed=0)
    hist = model["loss_history"]
    assert np.isfinite(hist[-1]) and hist[-1] < 0.5 * hist[0], (hist[0], hist[-1])
    keys = ("newton_its_sia", "newton_its_learned", "gmres_its_sia", "gmres_its_learned", "fallbacks")
    rep0 = evaluate(model, range(31000, 31008), n_points=500, fallback=0)
    rep1 = evaluate(model, range(31000, 31008), n_points=500, fallback=1)
    print("\n[learned, non-finite fallback]", {k: rep0[k] for k in keys})
    print("[learned, residual fallback]", {k: rep1[k] for k in keys})
    assert rep0["all_converged"] and rep1["all_converged"]
    for seed in range(31000, 31003):
        M = Mesh(learned_mesh(seed, n_points=500))
        Us = M.sia()
        U0, used0 = M.learned_guess(model["params"], model["norm"], fallback=0, smooth=2)
        U1, used1 = M.learned_guess(model["params"], model["norm"], fallback=1, smooth=2)
        assert used0 == 1 and bool(torch.isfinite(U0).all())
        n_nn = torch.linalg.vector_norm(M.residual(U0)).item()
        n_sia = torch.linalg.vector_norm(M.residual(Us)).item()
        if used1:
            assert n_nn <= n_sia * (1 + 1e-12) and torch.equal(U1, U0)
        else:
            assert n_nn >= n_sia * (1 - 1e-12) and torch.equal(U1, Us)
        M.close()


def test_committed_network_on_heldout_caps():
    """The committed network (the bench's learned-vs-plain line) on fixed held-out caps: it
    loads without pickling, every solve converges from either start, and the residual-checked
    guess keeps the network only where its residual norm is the smaller one.  The measured
    outcome on 200 held-out caps is that the learned start does not cut Newton time; the
    paired speedup on this subset is printed, not asserted."""
    import os
    from paper_2204_04321_amd import _lib
    from paper_2204_04321_amd.learned import evaluate, load_model
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2204_04321_amd", "weights", "learned_guess.npz")
    model = load_model(path)
    assert model["params"].numel() == int(_lib.lib().fo_mlp_param_count())
    assert model["norm"].numel() == 20 and model["adam_step"] > 0
    keys = ("newton_its_sia", "newton_its_learned", "speedup_geomean", "speedup_ci99", "fallbacks")
    for fb in (1, 0):
        rep = evaluate(model, range(20000, 20006), fallback=fb)
        print(f"\n[committed network, fallback {fb}]", {k: rep[k] for k in keys})
        assert rep["all_converged"]
        assert 0 <= rep["fallbacks"] <= 6
        if fb == 0:
            assert rep["fallbacks"] == 0
