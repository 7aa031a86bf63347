"""Train and evaluate the learned Newton initial guess on solutions the method generates.

    python -m paper_2204_04321_amd.learned --train 2000 --test 200 --out <dir>

Data: seeded ice caps (~2000 columns, 10 layers each) solved by fo_newton_solve from the
shallow-ice guess to ||F|| <= 1e-8 ||F(0)||; inputs are the library's column features,
targets asinh((u - u_sia) / 10 m/yr): the converged column profile as a correction of the
shallow-ice profile (which carries the rate factor A, absent from the features).  Training: the library's BF16
MLP forward/backward kernels, MSE and Adam, on the GPU.  Evaluation on held-out seeds:
Newton iterations, assembly calls and wall time from the learned guess (features,
inference and the fallback check included) against the shallow-ice guess, with the
speedup as exp(mean log-ratio) and a 99% t-interval over paired meshes (the paper's
Sec. 4.5 treatment of timing ratios).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from .api import MLP, Mesh

TOL = 1e-8


def _mesh(seed, n_points):
    from fo_inputs import learned_mesh
    return learned_mesh(seed, n_points=n_points)


def collect(seeds, n_points=2000, tol=TOL, verbose=False):
    """Solve every seed's mesh and gather (raw features, targets) on the device."""
    X, T, stats = [], [], []
    for i, seed in enumerate(seeds):
        desc = _mesh(seed, n_points)
        M = Mesh(desc)
        U = torch.zeros(M.n_dofs, dtype=torch.float64, device=M.device)
        rep = M.newton_solve(U, tol=tol, init="sia")
        if rep["status"] != 0:
            continue
        X.append(M.features())
        T.append(torch.asinh((U - M.sia()).view(M.n_verts, -1) / 10.0).float())
        stats.append(rep["newton_its"])
        if verbose and (i + 1) % 100 == 0:
            print(f"[collect] {i + 1} meshes, mean Newton its {np.mean(stats):.2f}", file=sys.stderr, flush=True)
        M.close()
    return {"X": torch.cat(X), "T": torch.cat(T), "newton_its": stats}


def train(data, epochs=30, batch=4096, lr=2e-3, seed=0, verbose=False):
    from ._lib import lib
    X, T = data["X"], data["T"]
    mean = X.mean(0)
    std = X.std(0) + 1e-6
    norm = torch.cat([mean, std]).float().contiguous()
    Xn = ((X - mean) / std).float().contiguous()
    g = torch.Generator(device="cpu").manual_seed(seed)
    rng = np.random.default_rng(seed)
    n = int(lib().fo_mlp_param_count())
    layers = MLP.LAYERS
    flat = []
    for i, j in zip(layers[:-1], layers[1:]):
        lim = math.sqrt(6.0 / (i + j))
        flat.append(rng.uniform(-lim, lim, i * j))
        flat.append(np.zeros(j))
    params = torch.from_numpy(np.concatenate(flat).astype(np.float32)).to(X.device)
    assert params.numel() == n
    net = MLP(params)
    N = Xn.shape[0]
    steps_per_epoch = max(1, N // batch)
    total = epochs * steps_per_epoch
    loss = torch.zeros(1, dtype=torch.float64, device=X.device)
    hist = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).to(X.device)
        loss.zero_()
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            xb = Xn.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            Y, acts = net.forward(xb)
            dY = MLP.mse_grad(Y, tb, loss)
            net.backward(xb, acts, dY)
            cur = lr * 0.5 * (1.0 + math.cos(math.pi * step / total))      # cosine decay
            net.adam(lr=cur)
            step += 1
        hist.append(loss.item() / steps_per_epoch)
        if verbose and (ep + 1) % max(1, epochs // 10) == 0:
            print(f"[train] epoch {ep + 1}/{epochs} mse {hist[-1]:.3e}", file=sys.stderr, flush=True)
    return {"params": net.params, "norm": norm, "loss_history": hist, "samples": N}


def evaluate(model, seeds, n_points=2000, tol=TOL, fallback=1, verbose=False):
    rows = []
    for k, seed in enumerate(seeds):
        if verbose and k and k % 50 == 0:
            print(f"[evaluate] {k} meshes", file=sys.stderr, flush=True)
        desc = _mesh(seed, n_points)
        M = Mesh(desc)
        ws = torch.empty(M.workspace_bytes(M.newton_opts()), dtype=torch.uint8, device=M.device)
        if k == 0:   # first-call effects out of the timings
            Uw = torch.zeros(M.n_dofs, dtype=torch.float64, device=M.device)
            M.newton_solve(Uw, workspace=ws, tol=tol, init="sia")
            M.learned_guess(model["params"], model["norm"], fallback=fallback)
        torch.cuda.synchronize()
        U = torch.zeros(M.n_dofs, dtype=torch.float64, device=M.device)
        t0 = time.perf_counter()
        rs = M.newton_solve(U, workspace=ws, tol=tol, init="sia")
        t_sia = time.perf_counter() - t0
        t0 = time.perf_counter()
        U2, used = M.learned_guess(model["params"], model["norm"], fallback=fallback)
        rl = M.newton_solve(U2, workspace=ws, tol=tol, init="user")
        t_l = time.perf_counter() - t0
        rows.append(dict(seed=seed, used_network=used, its_sia=rs["newton_its"], its_learned=rl["newton_its"],
                         lin_sia=rs["lin_its"], lin_learned=rl["lin_its"],
                         calls_sia=rs["residual_calls"] + rs["jacobian_calls"],
                         calls_learned=rl["residual_calls"] + rl["jacobian_calls"] + (2 if fallback else 0),
                         ok_sia=rs["status"] == 0, ok_learned=rl["status"] == 0,
                         t_sia=t_sia, t_learned=t_l))
        M.close()
    lr = np.log(np.array([r["t_sia"] / r["t_learned"] for r in rows]))
    n = len(rows)
    from scipy import stats as sps
    half = sps.t.ppf(0.995, n - 1) * lr.std(ddof=1) / math.sqrt(n) if n > 1 else float("nan")
    return {
        "fallback_rule": "non-finite or larger residual norm" if fallback else "non-finite only",
        "meshes": n,
        "newton_its_sia": int(sum(r["its_sia"] for r in rows)),
        "newton_its_learned": int(sum(r["its_learned"] for r in rows)),
        "gmres_its_sia": int(sum(r["lin_sia"] for r in rows)),
        "gmres_its_learned": int(sum(r["lin_learned"] for r in rows)),
        "assembly_calls_sia": int(sum(r["calls_sia"] for r in rows)),
        "assembly_calls_learned": int(sum(r["calls_learned"] for r in rows)),
        "wall_s_sia": float(sum(r["t_sia"] for r in rows)),
        "wall_s_learned": float(sum(r["t_learned"] for r in rows)),
        "speedup_geomean": float(math.exp(lr.mean())),
        "speedup_ci99": [float(math.exp(lr.mean() - half)), float(math.exp(lr.mean() + half))],
        "fallbacks": int(sum(1 for r in rows if not r["used_network"])),
        "all_converged": bool(all(r["ok_sia"] and r["ok_learned"] for r in rows)),
        "rows": rows,
    }


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--points", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--out", default="learned_out")
    a = ap.parse_args(argv)
    os.makedirs(a.out, exist_ok=True)
    t0 = time.perf_counter()
    data = collect(range(10000, 10000 + a.train), n_points=a.points, verbose=True)
    t_collect = time.perf_counter() - t0
    print(f"[learned] collected {data['X'].shape[0]} columns in {t_collect:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    model = train(data, epochs=a.epochs, batch=a.batch, verbose=True)
    t_train = time.perf_counter() - t0
    rep = evaluate(model, range(20000, 20000 + a.test), n_points=a.points, fallback=1, verbose=True)
    rep["without_residual_fallback"] = {k: v for k, v in evaluate(
        model, range(20000, 20000 + a.test), n_points=a.points, fallback=0, verbose=True).items() if k != "rows"}
    rep.update(train_meshes=a.train, train_columns=int(data["X"].shape[0]), epochs=a.epochs,
               final_train_mse=model["loss_history"][-1], collect_s=t_collect, train_s=t_train)
    np.savez(os.path.join(a.out, "model.npz"), params=model["params"].cpu().numpy(),
             norm=model["norm"].cpu().numpy())
    with open(os.path.join(a.out, "report.json"), "w") as f:
        json.dump(rep, f, indent=1)
    short = {k: v for k, v in rep.items() if k != "rows"}
    print(json.dumps(short))


if __name__ == "__main__":
    main()
