"""Train the warm-start network on generated graphs.

For each training graph (stochastic block model or Chung-Lu, alternating;
n ~ U[10k, 50k], mean degree ~ U[10, 30], Chung-Lu exponent ~ U[2.2, 2.8],
SBM blocks ~ U{5..50}; graph seed 1000 + i) the plain iSVD of
M = (1/K) sum_{j=1..K} T^j - lambda (11^T - A) gives the target top-k right
singular vectors (tolerance 1e-3), and isvd_ws_features gives the 16 node
features.  Training runs epochs of one Adam step per graph through
isvd_ws_train_step; all arithmetic is in the library's kernels.  The last
`--val` graphs are held out: after every epoch their mean loss (forward and
loss only, no update) is measured and the parameters of the best epoch are
kept.  Graph generation runs in host worker processes while the GPU computes
targets.

Writes <out>.npy (float32 parameter vector, the isvd_ws_get_params layout)
and <out>.json (training record).
"""

from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def graph_recipe(i: int):
    rng = np.random.default_rng(50_000 + i)
    n = int(rng.integers(10_000, 50_001))
    deg = float(rng.uniform(10.0, 30.0))
    if i % 2 == 0:
        return ("sbm", n, dict(num_blocks=int(rng.integers(5, 51)), mean_degree=deg, frac_in=0.77), 1000 + i)
    return ("chung_lu", n, dict(beta=float(rng.uniform(2.2, 2.8)), mean_degree=deg), 1000 + i)


def make_graph(i: int):
    from synth import chung_lu_graph, sbm_graph_by_degree
    kind, n, args, seed = graph_recipe(i)
    if kind == "sbm":
        g = sbm_graph_by_degree(n, seed=seed, **args)
    else:
        g = chung_lu_graph(n, seed=seed, **args)
    return i, kind, g


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--graphs", type=int, default=1000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--val", type=int, default=50)
    ap.add_argument("--k", type=int, default=128)
    ap.add_argument("--p", type=int, default=16)
    ap.add_argument("--K", type=int, default=10)
    ap.add_argument("--lam", type=float, default=0.1)
    ap.add_argument("--target-tol", type=float, default=1e-3)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2111_06312_amd", "weights", "warmstart_k128"))
    args = ap.parse_args()

    import torch

    from paper_2111_06312_amd import isvd as lib
    lib.load()
    coeffs = np.full(args.K, 1.0 / args.K)
    data = []
    t0 = time.time()
    ctx = mp.get_context("spawn")
    with ctx.Pool(args.workers) as pool:
        for i, kind, g in pool.imap(make_graph, range(args.graphs)):
            op = lib.Operator(g, form="ne", coeffs=coeffs, lam=args.lam, precision=lib.FP32)
            F = lib.features(op)
            _, _, V, info = op.truncated_svd(args.k, args.p, tol=args.target_tol, max_iter=600, seed=i,
                                             allow_not_converged=True)
            data.append((F, V.contiguous()))
            op.close()
            if i % 50 == 0:
                print(f"[train] target {i}: {kind} n={g.n} it={info.iterations} rho={info.residual:.1e} "
                      f"({time.time() - t0:.0f} s)", flush=True)
    t_data = time.time() - t0
    ws = lib.WarmStart(args.k, seed=args.seed)
    rng = np.random.default_rng(args.seed)
    ntrain = len(data) - args.val
    train, val = data[:ntrain], data[ntrain:]

    def val_loss():
        out = []
        for F, V in val:
            try:
                out.append(ws.train_step(F, V, lr=0.0)[0])
            except lib.IsvdError as e:
                if e.status != lib.ISVD_E_NOT_SPD:
                    raise
                out.append(1.0)       # rank-deficient output: no overlap credited
        return float(np.mean(out)) if out else float("nan")

    best = (val_loss(), -1, ws.get_params())
    print(f"[train] initial validation loss {best[0]:.4f}", flush=True)
    history, val_history = [], []
    for ep in range(args.epochs):
        order = rng.permutation(len(train))
        losses = []
        skipped = 0
        for j in order:
            F, V = train[j]
            try:
                loss, _ = ws.train_step(F, V, lr=args.lr)
            except lib.IsvdError as e:
                if e.status != lib.ISVD_E_NOT_SPD:
                    raise
                skipped += 1          # rank-deficient output: no update from this graph
                continue
            losses.append(loss)
        history.append(float(np.mean(losses)) if losses else float("nan"))
        val_history.append(val_loss())
        if val_history[-1] < best[0]:
            best = (val_history[-1], ep, ws.get_params())
        if skipped:
            print(f"[train] epoch {ep}: {skipped} steps skipped (rank-deficient output)", flush=True)
        print(f"[train] epoch {ep}: mean loss {history[-1]:.4f}, validation {val_history[-1]:.4f} "
              f"({time.time() - t0:.0f} s)", flush=True)
    torch.cuda.synchronize()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out + ".npy", best[2])
    with open(args.out + ".json", "w") as fh:
        json.dump({"k": args.k, "p": args.p, "K": args.K, "lambda": args.lam, "graphs": args.graphs,
                   "validation_graphs": args.val, "epochs": args.epochs, "lr": args.lr,
                   "target_tol": args.target_tol, "seed": args.seed, "best_epoch": best[1],
                   "best_validation_loss": best[0], "loss_per_epoch": history,
                   "validation_loss_per_epoch": val_history, "seconds_targets": round(t_data, 1),
                   "seconds_total": round(time.time() - t0, 1)}, fh, indent=1)
    print(f"[train] wrote {args.out}.npy", flush=True)


if __name__ == "__main__":
    main()
