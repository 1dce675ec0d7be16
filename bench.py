"""Benchmark of the BD3MG hot path on one MI355X.

A step is one BD3MG sweep (every block of the partition updated once: gradient,
direction, 2x2 solve and update passes for each colour of blocks) over the
256x256x64 FP32 workload (FP64 inner products, 2x2 solve and f): 200-ellipsoid
phantom, depth-variant Gaussian PSF 7x7x7 (sigma_xy 0.5 -> 3.0, sigma_z 1 -> 2),
noise 0.02, lambda = 0.01, delta = 0.02, eta = 0.01, 16 uneven blocks of 2..6
slices.  Inputs are synthetic and seeded; the observation y = H xbar + noise
is formed with the library's own H on the GPU.

Prints one JSON line: voxel-iterations/s over exactly --steps sweeps (after
--warmup untimed sweeps), the roofline figure of the dominant kernel (HIP
events on the library's stream, algorithmic bytes from the library), the
time to ||grad f|| / ||grad f(y)|| <= 1e-6 from x0 = y and from the learned
warm start x0 = y + net(y) (network inference inside the clock), the same
under the asynchronous-round schedule, and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-iterations/s + time-to-f-tolerance (plain vs warm-started), % HBM peak"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X vector FP32 (FP64: 78.6)
FP64_VALU_PEAK_TFLOPS = 78.6
WEIGHTS = os.path.join(ROOT, "paper_2002_02328_amd", "weights", "warmstart_c16.bin")


def net_flops(nvox, c=16):
    """Multiply-add flops of one forward pass of the warm-start U-Net (3x3x3
    convolutions at full, half and quarter resolution, 1x1x1 head)."""
    full = [(1, c), (c, c), (2 * c, c), (2 * c, c)]
    half = [(c, 2 * c), (2 * c, 2 * c), (4 * c, 2 * c), (4 * c, 2 * c)]
    quarter = [(2 * c, 4 * c), (4 * c, 4 * c)]
    per = sum(2 * 27 * a * b for a, b in full) + sum(2 * 27 * a * b for a, b in half) / 8.0 \
        + sum(2 * 27 * a * b for a, b in quarter) / 64.0 + 2 * c
    return per * nvox


def is_dense(w):
    return "psf" in w.extra


def make_problem(binding, w):
    nz, ny, nx = w.shape
    g = binding.Problem(nx, ny, nz, binding.FP64 if w.fp64 else binding.FP32)
    if is_dense(w):
        ps = w.extra["psf"]
        g.set_psf_dense(binding.psf_rotated_gaussian(ps["sx"], ps["sy"], ps["theta"], ps["sz"], w.kxy, w.kz))
    else:
        g.set_psf_gaussian(w.kxy, w.kz, w.sigma_xy, w.sigma_z)
    g.set_params(w.lam, w.delta, w.eta, w.kappa)
    y = g.H(w.xbar) + w.noise.astype(g.dtype)  # degradation model y = H xbar + b
    g.set_data(y.astype(g.dtype))
    g.set_blocks(w.nslices)
    return g


def dense_flops(w, ncolors, color):
    """Arithmetic of the general-kernel passes per sweep (one multiply and one
    add per kernel tap and output voxel, taps of the (2R+1)^2 in-slice
    planes): the gradient pass applies H^T on every block slice from the
    volume's slices within r_z, the direction pass H to d1 and d2 on S +- r_z
    of every block from the block's own slices within r_z."""
    nz, ny, nx = w.shape
    rz, R = w.kz // 2, max(w.kxy // 2, 1)
    tap = 2.0 * (2 * R + 1) ** 2 * nx * ny
    z0 = np.concatenate([[0], np.cumsum(w.nslices)[:-1]])
    grad = dirs = 0.0
    for b, n in enumerate(w.nslices):
        s0, s1 = int(z0[b]), int(z0[b] + n)
        for s in range(s0, s1):
            grad += (min(nz, s + rz + 1) - max(0, s - rz)) * tap
        for k in range(max(0, s0 - max(rz, 1 if w.kappa > 0 else 0)), min(nz, s1 + rz)):
            dirs += 2 * max(0, min(s1, k + rz + 1) - max(s0, k - rz)) * tap
    return {"grad": grad, "dirs": dirs}


def kernel_variant(w, kernel, tile_rows):
    """Name of the sweep kernel instance a pass runs, as the profiler prints it."""
    t = "double" if w.fp64 else "float"
    kz, r = w.kz, max(w.kxy // 2, 1)
    if is_dense(w):
        ty = tile_rows["dirs"]
        return {"grad": "k_dense<%s, %d, 1, true, %d>" % (t, r, ty), "dirs": "k_dense<%s, %d, 2, false, %d>" % (t, r, ty),
                "solve": "k_solve", "update": "k_dense_update<%s>" % t}[kernel]
    return {"grad": "k_grad<%s, %d>" % (t, kz),
            "dirs": "k_dirs<%s, %d, %d, %d>" % (t, kz, r, tile_rows["dirs"]),
            "solve": "k_solve",
            "update": "k_update<%s, %d, %d, false>" % (t, r, tile_rows["update"])}[kernel]


def measured_traffic(workload, variant):
    """HBM bytes per launch of a sweep kernel instance from the committed PMC
    record (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel calibration),
    or None when the kernel sources differ from those measured or the instance
    was not measured."""
    path = os.path.join(ROOT, "profiles", "traffic_sweep.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path)).get(workload)
    if not rec:
        return None
    h = hashlib.sha256()
    for f in ("bd3mg_kernels.hip", "bd3mg_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2002_02328_amd", "csrc", f), "rb").read())
    if h.hexdigest() != rec["kernel_source_sha256"]:
        return None
    return rec["bytes_per_launch"].get(variant)


def cpu_baseline(w, budget_s):
    """FP64 oracle on the same workload: as many whole sweeps as fit the budget."""
    import oracle
    if is_dense(w):
        ps = w.extra["psf"]
        pk = oracle.rotated_gauss_kernels(ps["sx"], ps["sy"], ps["theta"], ps["sz"], w.kxy, w.kz)
        y = oracle.Problem.with_kernels(np.zeros(w.shape), pk).H(w.xbar) + w.noise
        o = oracle.Problem.with_kernels(y, pk, lam=w.lam, delta=w.delta, eta=w.eta, kappa=w.kappa)
    else:
        gxy = oracle.gauss_table(w.sigma_xy, w.kxy)
        gz = oracle.gauss_table(w.sigma_z, w.kz)
        y = oracle.Problem(np.zeros(w.shape), gxy, gxy, gz).H(w.xbar) + w.noise
        o = oracle.Problem(y, gxy, gxy, gz, lam=w.lam, delta=w.delta, eta=w.eta, kappa=w.kappa)
    nc, order, _ = oracle.color_schedule(w.nslices, 2 * (w.kz // 2))
    x = y.copy()
    d = np.zeros(w.shape)
    t0 = time.perf_counter()
    o.run(x, d, w.nslices, order, 1, history=False)
    t1 = time.perf_counter()
    per = t1 - t0
    more = max(0, int(budget_s / per) - 1)
    if more:
        o.run(x, d, w.nslices, order, more, history=False)
    t2 = time.perf_counter()
    sweeps = 1 + more
    nvox = int(np.prod(w.shape))
    return {"value": nvox * sweeps / (t2 - t0), "unit": "voxel-iterations/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "%d sweeps of the %s workload from x0 = y (FP64, coloured order)"
                      % (sweeps, w.name),
            "seconds": t2 - t0}


def round_schedule(binding, w, args):
    """The same workload under asynchronous rounds (every block steps from one
    snapshot; one gradient, direction, solve and update launch per sweep) with
    the paper's majorant (no inflation): sweep throughput, per-kernel device
    time, and time to the tolerance from x0 = y and from the warm start."""
    nvox = int(np.prod(w.shape))
    r = make_problem(binding, w)
    r.set_blocks(w.nslices, binding.SCHED_ROUND)
    r.set_x0(None)
    (td, tu), _ = r.autotune(5)
    r.set_x0(None)
    r.run(args.warmup, check_every=0)
    t0 = time.perf_counter()
    r.run(args.steps, check_every=0)
    secs = time.perf_counter() - t0
    r.set_option(binding.OPT_PROFILE, 1)
    r.run(args.steps, check_every=0)
    prof = r.get_profile(reset=True)
    r.set_option(binding.OPT_PROFILE, 0)
    kernels = {k: {"launches": v[0], "avg_us": 1e3 * v[1] / max(v[0], 1),
                   "GB/s": (v[2] / (v[1] * 1e-3) / 1e9) if v[1] > 0 else None}
               for k, v in prof.items() if v[0] > 0 and k != "eval"}
    out = {"value": nvox * args.steps / secs, "unit": "voxel-iterations/s",
           "ms_per_step": 1e3 * secs / args.steps, "mu": 0.0, "tile_rows": {"dirs": td, "update": tu},
           "kernels": kernels, "lipschitz_bound": r.lipschitz_bound()}
    if not args.no_tol:
        def to_tol(net):
            r.set_x0(None)
            t0 = time.perf_counter()
            if net is not None:
                net.infer(r)
            res = r.run(args.max_sweeps_to_tol, grad_rtol=args.tol, check_every=1)
            return {"seconds": time.perf_counter() - t0, "sweeps": res["sweeps"],
                    "converged": bool(res["converged"]), "grad_rel": res["grad_norm"] / res["grad_norm_ref"],
                    "f": res["f"], "tol": args.tol}
        tt = {"plain_x0_y": to_tol(None), "warm_started": None}
        if os.path.exists(WEIGHTS) and not is_dense(w):
            net = binding.Net()
            net.load(open(WEIGHTS, "rb").read())
            net.infer(r)
            tt["warm_started"] = to_tol(net)
            net.close()
        out["time_to_tol"] = tt
    r.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="plain-fp32-256x256x64")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--max-sweeps-to-tol", type=int, default=20000)
    ap.add_argument("--no-tol", action="store_true", help="skip the time-to-tolerance run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-round", action="store_true", help="skip the asynchronous-round schedule")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (one GPU's share of the volume); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    from paper_2002_02328_amd import binding, inputs
    w = inputs.WORKLOADS[args.workload]()
    nvox = int(np.prod(w.shape))
    g = make_problem(binding, w)
    nc, order, color = g.get_schedule()

    # tile heights picked by the autotuner on this problem (state is restored)
    g.set_x0(None)
    (td, tu), tuned_ms = g.autotune(5)

    # timed sweeps
    g.set_x0(None)
    g.run(args.warmup, check_every=0)
    t0 = time.perf_counter()
    g.run(args.steps, check_every=0)  # returns after the device has finished
    t1 = time.perf_counter()
    secs = t1 - t0
    value = nvox * args.steps / secs

    # per-kernel device time over the same number of sweeps, events on the library's stream
    g.set_option(binding.OPT_PROFILE, 1)
    g.run(args.steps, check_every=0)
    prof = g.get_profile(reset=True)
    g.set_option(binding.OPT_PROFILE, 0)
    hot = {k: v for k, v in prof.items() if k != "eval" and v[0] > 0}
    dom = max(hot, key=lambda k: hot[k][1])
    variant = kernel_variant(w, dom, {"dirs": td, "update": tu})
    n, ms, by = hot[dom]
    achieved = by / (ms * 1e-3) / 1e9
    if is_dense(w):
        # the general-kernel passes are bound by vector arithmetic
        fl = dense_flops(w, nc, color)
        peak = FP64_VALU_PEAK_TFLOPS if w.fp64 else FP32_VALU_PEAK_TFLOPS
        tf = fl[dom] / (ms * 1e-3 / args.steps) / 1e12 if dom in fl else 0.0
        roof = {"bound": "alu", "kernel": dom, "variant": variant, "achieved": tf, "peak": peak,
                "unit": "TFLOP/s", "frac": tf / peak, "traffic": measured_traffic(w.name, variant),
                "avg_launch_us": 1e3 * ms / n, "flop_per_launch": fl.get(dom, 0.0) * args.steps / n,
                "flop_per_sweep": fl}
    else:
        roof = {"bound": "hbm", "kernel": dom, "variant": variant, "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(w.name, variant),
                "avg_launch_us": 1e3 * ms / n, "bytes_per_launch": by / n}
    kernels = {k: {"launches": v[0], "avg_us": 1e3 * v[1] / max(v[0], 1),
                   "GB/s": (v[2] / (v[1] * 1e-3) / 1e9) if v[1] > 0 else None}
               for k, v in prof.items() if v[0] > 0}
    total_ms = sum(v[1] for v in hot.values())
    all_bytes = sum(v[2] for v in hot.values())

    probe_gbs, _ = binding.probe_copy(4 << 30, 5)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * secs / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w.fp64 else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "shape_zyx": list(w.shape),
                   "psf": ("rotated %dx%dx%d" if is_dense(w) else "%dx%dx%d") % (w.kxy, w.kxy, w.kz),
                   "blocks": int(len(w.nslices)), "colors": int(nc),
                   "reductions": "f64", "step": "one sweep (every block updated once)",
                   "tile_rows": {"dirs": td, "update": tu}},
        "roofline": roof,
        "kernels": kernels,
        "sweep_algorithmic_GBps": all_bytes / (total_ms * 1e-3) / 1e9,
        "copy_probe_GBps": probe_gbs,
    }

    if not args.no_tol:
        net = None
        if os.path.exists(WEIGHTS) and not is_dense(w):  # trained on the separable-blur volumes
            net = binding.Net()
            net.load(open(WEIGHTS, "rb").read())
            net.infer(g)  # sizes the network's buffers for this volume (untimed)

        def to_tol(tol, warm):
            g.set_x0(None)
            t0 = time.perf_counter()
            if warm:
                net.infer(g)  # x0 = y + net(y), inside the clock
            res = g.run(args.max_sweeps_to_tol, grad_rtol=tol, check_every=1)
            t1 = time.perf_counter()
            return {"seconds": t1 - t0, "sweeps": res["sweeps"], "converged": bool(res["converged"]),
                    "grad_rel": res["grad_norm"] / res["grad_norm_ref"], "f": res["f"], "tol": tol}

        tt = {"plain_x0_y": to_tol(args.tol, False), "warm_started": None}
        if net is not None:
            tt["warm_started"] = to_tol(args.tol, True)
            tt["speedup"] = tt["plain_x0_y"]["seconds"] / tt["warm_started"]["seconds"]
            loose = {"plain_x0_y": to_tol(1e-4, False), "warm_started": to_tol(1e-4, True)}
            loose["speedup"] = loose["plain_x0_y"]["seconds"] / loose["warm_started"]["seconds"]
            tt["at_1e-4"] = loose
            # network inference alone (bf16 matrix cores), averaged over repeats
            reps = 10
            t0 = time.perf_counter()
            for _ in range(reps):
                net.infer(g)
            ms = 1e3 * (time.perf_counter() - t0) / reps
            flop = net_flops(nvox)
            tt["inference"] = {"ms": ms, "TFLOP/s": flop / (ms * 1e-3) / 1e12,
                               "frac_bf16_peak": flop / (ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
                               "flop": flop, "weights": os.path.relpath(WEIGHTS, ROOT)}
            net.close()
        out["time_to_tol"] = tt

    if not args.no_round:
        out["round_schedule"] = round_schedule(binding, w, args)

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
