"""Learned warm start: training data, training and deployment of the network.

Training tiles are 256 x 256 random metasurfaces with their own 20-cell PML,
generated as the 1024 x 1024 benchmark grid but with 16 pillars (see
workloads.learned.tile_workload); each is solved by this library (complex64
fronts, FP64 FGMRES to rel-res 1e-8) and its (features, field) pair taken by
stf_nn_tile_data.  Training runs the library's own forward/backward/Adam
kernels (stf_nn_train_step).  Deployment: Problem.solve(..., x0="learned")
with the network attached to the context.

    python -m paper_2509_20801_amd.learned --tiles 4000 --epochs 24 --out weights.npz
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

DEFAULT = dict(n=256, width=16, modes=16, layers=4, cin=3)
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "nn_metasurface_256.npz")


def _prm(p, prec):
    return dict(nx=p["nx"], ny=p["ny"], k0=p["k0"], pml=p["pml"], pml_order=p["pml_order"],
                pml_R=p["pml_R"], px=p["px"], py=p["py"], overlap=p["overlap"],
                local_pml=p["local_pml"], local_pml_order=p["local_pml_order"],
                local_pml_R=p["local_pml_R"], front_prec=prec)


def generate(stf, ctx, net, n_tiles, seed0=50000, subcells=4, tol=1e-8, log=print):
    """(features, fields) float32 CUDA tensors (n_tiles, 3|2, n, n) from plain-method solves."""
    import torch
    from workloads import learned as wl
    n = net.cfg.n
    f = torch.empty((n_tiles, 3, n, n), dtype=torch.float32, device="cuda")
    t = torch.empty((n_tiles, 2, n, n), dtype=torch.float32, device="cuda")
    pb = None
    iters = []
    t0 = time.time()
    for i in range(n_tiles):
        w = wl.tile_workload(seed0 + i, interior=n, subcells=subcells)
        eps = torch.from_numpy(w.eps_cells).cuda()
        b = torch.from_numpy(w.b[0]).cuda()
        if pb is None:
            pb = stf.Problem(ctx, _prm(w.params(), stf.STF_C64), eps)
        else:
            pb.assemble(eps)
        pb.factor()
        x, info = pb.solve(b, tol=tol, restart=20, max_iter=400)
        iters.append(info[0]["iters"])
        fi, ti = pb.tile_data(net, b, x)
        f[i].copy_(fi[0])
        t[i].copy_(ti[0])
        if (i + 1) % 250 == 0 or i + 1 == n_tiles:
            log("tiles %d/%d  %.1f s  mean iters %.1f" % (i + 1, n_tiles, time.time() - t0,
                                                          float(np.mean(iters))))
    if pb is not None:
        pb.close()
    return f, t


def train(net, f, t, epochs, batch, lr, seed=0, holdout=0, log=print):
    """Adam on mini-batches of a fixed random order of the tiles; cosine decay of
    the learning rate.  Returns the per-epoch mean training loss (and the
    hold-out loss when holdout > 0: the last `holdout` tiles are not trained on)."""
    rng = np.random.default_rng(seed)
    N = int(f.shape[0]) - holdout
    nb = N // batch
    steps = epochs * nb
    hist = []
    step = 0
    t0 = time.time()
    for e in range(epochs):
        order = rng.permutation(nb)
        tot = 0.0
        for k in order:
            step += 1
            a = lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / steps))
            s = slice(int(k) * batch, int(k + 1) * batch)
            tot += net.train_step(f[s], t[s], a, step)
        rec = {"epoch": e + 1, "train_loss": tot / nb, "seconds": time.time() - t0}
        if holdout:
            hl = 0.0
            for j in range(N, N + holdout, batch):
                s = slice(j, min(j + batch, N + holdout))
                hl += net.loss_grad(f[s], t[s])[0] * (s.stop - s.start)
            rec["holdout_loss"] = hl / holdout
        hist.append(rec)
        log(json.dumps(rec))
    return hist


def evaluate(stf, ctx, net, w, prec=None, tol=1e-8, restart=20, max_iter=600, log=print):
    """Iterations and wall time of the solve of workload w from the zero guess
    and from the learned guess (factorisation excluded, same factors)."""
    import torch
    prec = stf.STF_C64 if prec is None else prec
    eps = torch.from_numpy(w.eps_cells).cuda()
    b = torch.from_numpy(w.b[0]).cuda()
    pb = stf.Problem(ctx, _prm(w.params(), prec), eps)
    pb.factor()
    ctx.set_nn(net)
    out = {"workload": w.name, "ndof": w.nx * w.ny}
    for mode in ("zero", "learned", "zero", "learned"):       # second pass timed warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, inf = pb.solve(b, tol=tol, restart=restart, max_iter=max_iter,
                          x0="learned" if mode == "learned" else None)
        torch.cuda.synchronize()
        out[mode] = {"iters": inf[0]["iters"], "seconds": round(time.perf_counter() - t0, 4),
                     "relres_true": inf[0]["relres_true"], "relres_x0": inf[0]["relres_x0"],
                     "used_learned": inf[0]["used_learned"]}
    ctx.set_nn(None)
    pb.close()
    log(json.dumps(out))
    return out


def load_network(stf, ctx, path=WEIGHTS, max_batch=16):
    """The trained network stored at `path` (None if the file is absent)."""
    if not os.path.exists(path):
        return None
    z = np.load(path, allow_pickle=False)
    cfg = {k: int(z[k]) for k in ("n", "width", "modes", "layers", "cin")}
    return stf.Network(ctx, z["params"], max_batch=max_batch, **cfg)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--tiles", type=int, default=4000)
    ap.add_argument("--holdout", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=24)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--eval", action="store_true", help="evaluate on the 1024^2 and 2048^2 grids")
    args = ap.parse_args()
    import torch  # noqa: F401
    import paper_2509_20801_amd as stf
    from workloads import learned as wl

    def log(s):
        print(s, flush=True)

    ctx = stf.Context(0)
    flat = wl.init_params(DEFAULT["width"], DEFAULT["modes"], DEFAULT["layers"], DEFAULT["cin"],
                          args.seed)
    net = stf.Network(ctx, flat, max_batch=args.batch, **DEFAULT)
    t0 = time.time()
    f, t = generate(stf, ctx, net, args.tiles, log=log)
    t_gen = time.time() - t0
    t0 = time.time()
    hist = train(net, f, t, args.epochs, args.batch, args.lr, args.seed, args.holdout, log=log)
    t_train = time.time() - t0
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.savez_compressed(args.out, params=net.get_params(), history=json.dumps(hist),
                        gen_seconds=t_gen, train_seconds=t_train, tiles=args.tiles,
                        epochs=args.epochs, **DEFAULT)
    log(json.dumps({"saved": args.out, "gen_s": round(t_gen, 1), "train_s": round(t_train, 1),
                    "final": hist[-1]}))
    if args.eval:
        from workloads import configs
        evaluate(stf, ctx, net, configs.metasurface_sheet(interior=1024, parts=8, seed=5001), log=log)
        evaluate(stf, ctx, net, configs.metasurface_sheet(interior=2048, parts=16, seed=5002), log=log)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
