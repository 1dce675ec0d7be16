"""Train the learned warm start x0 = y + net(y) on pairs (y, x*) that the
library itself produces: seeded 128x128x32 volumes (inputs.warmstart_train_member)
are blurred with the library's H, solved in batches with BD3MG to the
tolerance the workloads are run to (1e-6 of ||grad f(y)|| by default), and
the network is fitted to the solutions with the library's Adam step.  The
time to tolerance from y and from y + net(y) is then measured on the eight
held-out 256x256x64 volumes and the benchmark's volume, at 1e-4 and 1e-6.
Everything runs through libbd3mg; this script only marshals arrays.

Usage:
  python -m paper_2002_02328_amd.train_warmstart --pairs 2000 --epochs 20 \
      --out paper_2002_02328_amd/weights/warmstart_c16.bin --log train.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2002_02328_amd import binding, inputs  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "warmstart_c16.bin")


def make_problem(w):
    nz, ny, nx = w.shape
    p = binding.Problem(nx, ny, nz, binding.FP32)
    p.set_psf_gaussian(w.kxy, w.kz, w.sigma_xy, w.sigma_z)
    p.set_params(w.lam, w.delta, w.eta, w.kappa)
    y = (p.H(w.xbar) + w.noise).astype(np.float32)  # y = H xbar + noise
    p.set_data(y)
    p.set_blocks(w.nslices)
    p.set_x0(None)
    return p, y


def make_pairs(n, tol, max_sweeps, group=16, log=print):
    shape = inputs.warmstart_train_member(0).shape
    ys = np.empty((n,) + shape, np.float32)
    xs = np.empty((n,) + shape, np.float32)
    sweeps = []
    t0 = time.perf_counter()
    for g0 in range(0, n, group):
        ids = list(range(g0, min(n, g0 + group)))
        probs = []
        for t in ids:
            p, y = make_problem(inputs.warmstart_train_member(t))
            ys[t] = y
            probs.append(p)
        b = binding.Batch(probs)
        res = b.run(max_sweeps, grad_rtol=tol, check_every=8)
        for t, p, r in zip(ids, probs, res):
            xs[t] = p.get_x()
            sweeps.append(r["sweeps"])
        b.close()
        for p in probs:
            p.close()
        if (g0 // group) % 10 == 0:
            log("pairs %d/%d  mean sweeps %.0f  %.1f s" % (ids[-1] + 1, n, np.mean(sweeps), time.perf_counter() - t0))
    return ys, xs, {"seconds": time.perf_counter() - t0, "sweeps_mean": float(np.mean(sweeps)),
                    "sweeps_max": int(np.max(sweeps)), "tol": tol}


def mse(a, b):
    return float(np.mean((a.astype(np.float64) - b.astype(np.float64)) ** 2))


def train(net, ys, xs, epochs, batch, lr0, lr1, nval, seed, log=print):
    n = ys.shape[0]
    ntr = n - nval
    rng = np.random.default_rng(seed)
    per_epoch = ntr // batch
    total = epochs * per_epoch
    hist = []
    k = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = rng.permutation(ntr)
        run = []
        for i in range(per_epoch):
            idx = np.sort(perm[i * batch:(i + 1) * batch])
            lr = lr1 + 0.5 * (lr0 - lr1) * (1 + math.cos(math.pi * k / max(1, total - 1)))
            loss = net.train_step(ys[idx], xs[idx], lr, want_loss=True)
            run.append(loss)
            k += 1
        val = evaluate(net, ys[ntr:], xs[ntr:]) if nval else None
        hist.append({"epoch": ep, "train_loss": float(np.mean(run)), "val": val,
                     "seconds": time.perf_counter() - t0})
        log("epoch %d  train mse %.3e  val %s  %.1f s" % (ep, np.mean(run), val, time.perf_counter() - t0))
    return hist, {"steps": k, "seconds": time.perf_counter() - t0, "batch": batch}


def evaluate(net, ys, xs, batch=8):
    """MSE of x0 = y + net(y) and of x0 = y against the solutions."""
    e_net, e_y = 0.0, 0.0
    for i in range(0, ys.shape[0], batch):
        x0 = net.forward(ys[i:i + batch])
        e_net += mse(x0, xs[i:i + batch]) * x0.shape[0]
        e_y += mse(ys[i:i + batch], xs[i:i + batch]) * x0.shape[0]
    return {"mse_net": e_net / ys.shape[0], "mse_y": e_y / ys.shape[0]}


def time_to_tol(w, net=None, tol=1e-6, max_sweeps=20000, tiles=None):
    """Seconds and sweeps from x0 = y (net None) or x0 = y + net(y) (inference
    inside the clock) to ||grad f|| <= tol ||grad f(y)||, checked every sweep."""
    nz, ny, nx = w.shape
    p = binding.Problem(nx, ny, nz, binding.FP32)
    p.set_psf_gaussian(w.kxy, w.kz, w.sigma_xy, w.sigma_z)
    p.set_params(w.lam, w.delta, w.eta, w.kappa)
    y = (p.H(w.xbar) + w.noise).astype(np.float32)
    p.set_data(y)
    p.set_blocks(w.nslices)
    p.set_x0(None)
    if tiles is None:
        tiles, _ = p.autotune(5)
    else:
        p.set_option(binding.OPT_TILE_ROWS_DIRS, tiles[0])
        p.set_option(binding.OPT_TILE_ROWS_UPDATE, tiles[1])
    p.set_x0(None)
    t0 = time.perf_counter()
    if net is not None:
        net.infer(p)
    t_inf = time.perf_counter() - t0
    res = p.run(max_sweeps, grad_rtol=tol, check_every=1)
    t1 = time.perf_counter()
    out = {"seconds": t1 - t0, "infer_seconds": t_inf, "sweeps": res["sweeps"],
           "converged": bool(res["converged"]), "grad_rel": res["grad_norm"] / res["grad_norm_ref"],
           "f": res["f"], "tol": tol, "tile_rows": list(tiles)}
    p.close()
    return out


def eval_volumes(n):
    """The n held-out 256x256x64 volumes, then the benchmark's own volume."""
    return [(w.name + "-eval%d" % e, w) for e, w in ((e, inputs.warmstart_eval_member(e)) for e in range(n))] + \
        [(inputs.mid_fp32().name, inputs.mid_fp32())]


def gain(net, volumes, tols=(1e-4, 1e-6), log=print):
    rows = []
    for name, w in eval_volumes(volumes):
        for tol in tols:
            plain = time_to_tol(w, None, tol)
            warm = time_to_tol(w, net, tol, tiles=plain["tile_rows"])
            rows.append({"volume": name, "tol": tol, "plain": plain, "warm": warm,
                         "speedup": plain["seconds"] / warm["seconds"]})
            log("%s tol %.0e: plain %d sweeps %.3f s, warm %d sweeps %.3f s (inference %.4f s)"
                % (name, tol, plain["sweeps"], plain["seconds"], warm["sweeps"], warm["seconds"],
                   warm["infer_seconds"]))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=2000)
    ap.add_argument("--val", type=int, default=100)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-sweeps", type=int, default=20000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--lr-end", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--log", default=None)
    ap.add_argument("--eval", type=int, default=8,
                    help="held-out 256x256x64 volumes for the time-to-tolerance gain (the benchmark's is added)")
    args = ap.parse_args()

    def log(msg):
        print(msg, flush=True)

    ys, xs, gen = make_pairs(args.pairs, args.tol, args.max_sweeps, log=log)
    log("pairs ready: %s" % gen)
    net = binding.Net()
    net.set_params(inputs.net_init_params(args.seed, head_scale=0.1).astype(np.float32))
    hist, tr = train(net, ys, xs, args.epochs, args.batch, args.lr, args.lr_end, args.val, args.seed, log=log)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "wb") as fh:
        fh.write(net.save())
    log("wrote %s" % args.out)
    rows = gain(net, args.eval, log=log) if args.eval >= 0 else []
    if args.log:
        with open(args.log, "w") as fh:
            json.dump({"command": "python -m paper_2002_02328_amd.train_warmstart " + " ".join(sys.argv[1:]),
                       "args": vars(args), "pairs": gen, "train": tr, "history": hist, "gain": rows}, fh, indent=1)


if __name__ == "__main__":
    main()
