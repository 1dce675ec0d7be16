"""Write the stored expected values of the full-size parity tests.

Calls only the FP64 oracle (oracle/) and the seeded input generator.  For the
256x256x64 workload (y and PSF factors rounded to FP32 once, as both sides use
them) it runs the oracle's BD3MG until ||grad f|| <= tol ||grad f(y)||, then
records the minimiser: f*, ||x*||, the gradient ratio reached, and x* at a
seeded sample of voxels; plus the FP32 floor, ||grad f(fl32(x*))|| /
||grad f(y)||.  Output: tests/golden/plain_fp32_256x256x64.json.

Usage: python tests/golden/make_golden.py [--tol 1e-10] [--chunk 200]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2002_02328_amd import inputs  # noqa: E402

NSAMPLE = 4096
SAMPLE_SEED = 777


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--chunk", type=int, default=200)
    ap.add_argument("--max-sweeps", type=int, default=40000)
    ap.add_argument("--save-x", default=None, help="also save x* as .npy here")
    args = ap.parse_args()

    w = inputs.mid_fp32()
    gxy = f32(oracle.gauss_table(w.sigma_xy, w.kxy))
    gz = f32(oracle.gauss_table(w.sigma_z, w.kz))
    y = f32(oracle.Problem(np.zeros(w.shape), gxy, gxy, gz).H(w.xbar) + w.noise)
    p = oracle.Problem(y, gxy, gxy, gz, lam=w.lam, delta=w.delta, eta=w.eta, kappa=w.kappa)
    nc, order, _ = oracle.color_schedule(w.nslices, 2 * p.rz)
    g0 = p.grad_norm(y)
    x = y.copy()
    d = np.zeros(w.shape)
    sweeps = 0
    t0 = time.time()
    ratio = 1.0
    hist = []
    while sweeps < args.max_sweeps:
        p.run(x, d, w.nslices, order, args.chunk, history=False)
        sweeps += args.chunk
        ratio = p.grad_norm(x) / g0
        hist.append([sweeps, ratio])
        print("sweeps %d  ||grad f||/||grad f(y)|| = %.3e  (%.0f s)" % (sweeps, ratio, time.time() - t0),
              flush=True)
        if ratio <= args.tol:
            break
    fstar = p.f(x)
    floor = p.grad_norm(f32(x)) / g0
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = np.sort(rng.choice(x.size, size=NSAMPLE, replace=False))
    out = {
        "workload": w.name,
        "note": "FP64 oracle, coloured order, y and PSF factors rounded to FP32",
        "sweeps": sweeps,
        "grad_ratio": ratio,
        "grad_ref": g0,
        "f_star": fstar,
        "x_norm": float(np.linalg.norm(x)),
        "fp32_floor_grad_ratio": floor,
        "sample_seed": SAMPLE_SEED,
        "sample_index": idx.tolist(),
        "sample_x": [float(v) for v in x.ravel()[idx]],
        "history": hist,
    }
    path = os.path.join(ROOT, "tests", "golden", "plain_fp32_256x256x64.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    if args.save_x:
        np.save(args.save_x, x)
    print("wrote", path, "f* = %.12g, floor = %.3e" % (fstar, floor))


if __name__ == "__main__":
    main()
