"""Seeded synthetic workloads for BD3MG deblurring.

This module only draws inputs: the phantom volume, the noise field, the
per-slice blur widths, the block partition and the criterion's parameters.
It holds none of the method's arithmetic (no PSF tables, no blur, no
criterion), so both the HIP library and the CPU oracle can consume the same
draws.  The observation y = H xbar + noise is formed by whichever side owns an
H (the oracle in tests, the library in the benchmark).

The paper's volumes (FlyBrain 256x256x24 and Aneurysm 155x154x79, Sec. 3.2 and
3.3) are not available; seeded ellipsoid phantoms of the same kind of content
(piecewise-constant objects in [0, 1]) stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    name: str
    shape: tuple            # (nz, ny, nx)
    xbar: np.ndarray        # phantom, float64 in [0, 1]
    noise: np.ndarray       # sigma_n * N(0, 1), float64, x fastest
    sigma_xy: np.ndarray    # [nz] Gaussian width in x and y for each depth
    sigma_z: np.ndarray     # [nz] Gaussian width along z for each depth
    kxy: int                # kernel size in x and y (odd)
    kz: int                 # kernel size in z (odd)
    lam: float
    delta: float
    eta: float
    kappa: float
    nslices: np.ndarray     # block partition along z (slice counts)
    sweeps: int = 0         # fixed sweep count of the workload (0: run to tolerance)
    grad_rtol: float = 0.0  # stop when ||grad f|| <= grad_rtol * ||grad f(y)||
    fp64: bool = False      # storage precision of the workload
    extra: dict = field(default_factory=dict)


def ellipsoid_phantom(shape, n_ellipsoids, rng, axes=(3.0, 15.0), vals=(0.2, 1.0)):
    """Sum of axis-aligned ellipsoids, clipped to [0, 1].

    Per ellipsoid the draws are, in order: centre (cx, cy, cz) uniform over the
    volume's index range, semi-axes (ax, ay, az) ~ U[axes], intensity ~ U[vals].
    Voxel (i, j, k) is inside when ((i-cx)/ax)^2 + ((j-cy)/ay)^2 + ((k-cz)/az)^2 <= 1.
    """
    nz, ny, nx = shape
    vol = np.zeros(shape, dtype=np.float64)
    for _ in range(int(n_ellipsoids)):
        cx = rng.uniform(0.0, nx - 1)
        cy = rng.uniform(0.0, ny - 1)
        cz = rng.uniform(0.0, nz - 1)
        ax = rng.uniform(*axes)
        ay = rng.uniform(*axes)
        az = rng.uniform(*axes)
        v = rng.uniform(*vals)
        i0, i1 = max(0, int(np.floor(cx - ax))), min(nx - 1, int(np.ceil(cx + ax)))
        j0, j1 = max(0, int(np.floor(cy - ay))), min(ny - 1, int(np.ceil(cy + ay)))
        k0, k1 = max(0, int(np.floor(cz - az))), min(nz - 1, int(np.ceil(cz + az)))
        if i0 > i1 or j0 > j1 or k0 > k1:
            continue
        ii = (np.arange(i0, i1 + 1) - cx) / ax
        jj = (np.arange(j0, j1 + 1) - cy) / ay
        kk = (np.arange(k0, k1 + 1) - cz) / az
        inside = (kk[:, None, None] ** 2 + jj[None, :, None] ** 2 + ii[None, None, :] ** 2) <= 1.0
        vol[k0:k1 + 1, j0:j1 + 1, i0:i1 + 1] += v * inside
    return np.clip(vol, 0.0, 1.0)


def linear_schedule(nz, start, end):
    """sigma(k) = start + (end - start) k / (nz - 1); constant when nz == 1."""
    if nz == 1:
        return np.array([float(start)])
    k = np.arange(nz, dtype=np.float64)
    return start + (end - start) * k / (nz - 1)


def uneven_partition(nz, nblocks, lo, hi, rng):
    """nblocks slice counts drawn uniformly in {lo..hi}, redrawn until they sum to nz."""
    if not (lo * nblocks <= nz <= hi * nblocks):
        raise ValueError("no partition of %d slices into %d blocks of %d..%d" % (nz, nblocks, lo, hi))
    while True:
        n = rng.integers(lo, hi + 1, size=nblocks)
        if int(n.sum()) == nz:
            return n.astype(np.int32)


def cut_partition(nz, nblocks, rng):
    """nblocks blocks of >= 1 slice from nblocks-1 distinct random cut points."""
    nblocks = min(nblocks, nz)
    cuts = np.sort(rng.choice(np.arange(1, nz), size=nblocks - 1, replace=False))
    edges = np.concatenate([[0], cuts, [nz]])
    return np.diff(edges).astype(np.int32)


def _seeds(base):
    return (np.random.default_rng(base + 1), np.random.default_rng(base + 2),
            np.random.default_rng(base + 3))


def paper_x0(y, seed):
    """The paper's starting point (Sec. 3.1, experimental setup): entries drawn
    uniformly in [0, max(y)], x fastest, from default_rng(seed)."""
    y = np.asarray(y)
    return np.random.default_rng(seed).uniform(0.0, float(np.max(y)), size=y.shape)


def small_plain_fp64(seed=1000):
    """64x64x16 FP64 volume, 20 ellipsoids, PSF 5x5x5 (sigma_xy 0.5 -> 2.0 over
    z, sigma_z = 1), noise 0.02, lambda 0.01, delta 0.02, eta 0.01, four blocks
    of four slices, 200 sweeps."""
    shape = (16, 64, 64)
    rp, rn, _ = _seeds(seed)
    xbar = ellipsoid_phantom(shape, 20, rp)
    noise = 0.02 * rn.standard_normal(shape)
    return Workload("plain-fp64-64x64x16", shape, xbar, noise,
                    linear_schedule(16, 0.5, 2.0), np.full(16, 1.0), 5, 5,
                    0.01, 0.02, 0.01, 0.0, np.array([4, 4, 4, 4], np.int32),
                    sweeps=200, fp64=True)


def mid_fp32(seed=2000):
    """256x256x64 FP32 volume, 200 ellipsoids, PSF 7x7x7 (sigma_xy 0.5 -> 3.0,
    sigma_z 1.0 -> 2.0), noise 0.02, lambda 0.01, delta 0.02, eta 0.01, 16 uneven
    blocks of 2..6 slices; run to ||grad f|| / ||grad f(y)|| < 1e-6."""
    shape = (64, 256, 256)
    rp, rn, rb = _seeds(seed)
    xbar = ellipsoid_phantom(shape, 200, rp)
    noise = 0.02 * rn.standard_normal(shape)
    return Workload("plain-fp32-256x256x64", shape, xbar, noise,
                    linear_schedule(64, 0.5, 3.0), linear_schedule(64, 1.0, 2.0), 7, 7,
                    0.01, 0.02, 0.01, 0.0, uneven_partition(64, 16, 2, 6, rb),
                    grad_rtol=1e-6)


def large_fp32(seed=3000):
    """512x512x128 FP32 volume, 1600 ellipsoids, PSF 9x9x9 (sigma_xy 0.5 -> 3.5,
    sigma_z 1.0 -> 2.0), noise 0.01, lambda 0.005, delta 0.01, eta 0.01, 32
    uneven blocks of 2..6 slices, 100 sweeps."""
    shape = (128, 512, 512)
    rp, rn, rb = _seeds(seed)
    xbar = ellipsoid_phantom(shape, 1600, rp)
    noise = 0.01 * rn.standard_normal(shape)
    return Workload("plain-fp32-512x512x128", shape, xbar, noise,
                    linear_schedule(128, 0.5, 3.5), linear_schedule(128, 1.0, 2.0), 9, 9,
                    0.005, 0.01, 0.01, 0.0, uneven_partition(128, 32, 2, 6, rb),
                    sweeps=100)


def batch_member(p, seed_base=4000):
    """Problem p of the batched workload: nx, ny ~ U{128..256}, nz ~ U{32..96},
    ellipsoid density of the 256x256x64 volume (at least 20), PSF 7x7x7 with its
    own sigma_xy range (start U[0.4, 0.8], end U[1.5, 3.0]), sigma_z 1 -> 2,
    noise U[0.01, 0.03], 4..16 blocks from random cuts."""
    base = seed_base + 10 * p
    rs = np.random.default_rng(base)
    nx = int(rs.integers(128, 257))
    ny = int(rs.integers(128, 257))
    nz = int(rs.integers(32, 97))
    s0 = rs.uniform(0.4, 0.8)
    s1 = rs.uniform(1.5, 3.0)
    sn = rs.uniform(0.01, 0.03)
    nb = int(rs.integers(4, 17))
    shape = (nz, ny, nx)
    rp, rn, rb = _seeds(base)
    ne = max(20, int(round(200 * nx * ny * nz / (256 * 256 * 64))))
    xbar = ellipsoid_phantom(shape, ne, rp)
    noise = sn * rn.standard_normal(shape)
    return Workload("batch-%d-%dx%dx%d" % (p, nx, ny, nz), shape, xbar, noise,
                    linear_schedule(nz, s0, s1), linear_schedule(nz, 1.0, 2.0), 7, 7,
                    0.01, 0.02, 0.01, 0.0, cut_partition(nz, nb, rb), sweeps=50)


def tiny(shape, seed, kxy=3, kz=3, nblocks=None, lam=0.01, delta=0.05, eta=0.01, kappa=0.0,
         sigma_xy=(0.5, 1.5), sigma_z=(0.6, 1.2), noise=0.02, n_ellipsoids=4):
    """Small random problem for tests: few ellipsoids sized to the volume."""
    nz, ny, nx = shape
    rp, rn, rb = _seeds(seed)
    amax = max(1.5, min(shape) / 2.0)
    xbar = ellipsoid_phantom(shape, n_ellipsoids, rp, axes=(1.0, amax))
    nz_ = shape[0]
    if nblocks is None:
        nblocks = max(1, nz_ // 2)
    nsl = cut_partition(nz_, nblocks, rb) if nblocks > 1 else np.array([nz_], np.int32)
    return Workload("tiny-%dx%dx%d" % (nx, ny, nz), shape, xbar, noise * rn.standard_normal(shape),
                    linear_schedule(nz, *sigma_xy), linear_schedule(nz, *sigma_z), kxy, kz,
                    lam, delta, eta, kappa, nsl, sweeps=10, fp64=True)


def rotated_psf_draws(nz, rng, sxy=(0.5, 2.5), sz=(1.0, 4.0)):
    """Per-depth parameters of a rotated anisotropic Gaussian blur (the paper
    draws variance and rotation per depth from uniform laws): in-slice widths
    sx, sy ~ U[sxy], rotation theta ~ U[0, pi), z width sz ~ U[sz]."""
    return {"sx": rng.uniform(*sxy, nz), "sy": rng.uniform(*sxy, nz),
            "theta": rng.uniform(0.0, np.pi, nz), "sz": rng.uniform(*sz, nz)}


def dense_fp32_256x256x24(seed=7000):
    """256x256x24 FP32 volume (the size of the paper's FlyBrain test), 60
    ellipsoids, per-depth rotated Gaussian kernels 11x11x21 (in-slice widths
    U[0.5, 2.5], rotation U[0, pi), z width U[1, 4]), noise 0.04, lambda 0.01,
    delta 0.02, eta 0.01, 8 uneven blocks of 2..4 slices."""
    shape = (24, 256, 256)
    rp, rn, rb = _seeds(seed)
    xbar = ellipsoid_phantom(shape, 60, rp)
    noise = 0.04 * rn.standard_normal(shape)
    psf = rotated_psf_draws(24, np.random.default_rng(seed + 3))
    return Workload("dense-fp32-256x256x24", shape, xbar, noise, np.zeros(24), np.zeros(24), 11, 21,
                    0.01, 0.02, 0.01, 0.0, uneven_partition(24, 8, 2, 4, rb), grad_rtol=1e-4,
                    extra={"psf": psf})


def dense_fp32_155x154x79(seed=7100):
    """155x154x79 FP32 volume (the size of the paper's Aneurysm test), 80
    ellipsoids, per-depth rotated Gaussian kernels 5x5x11 (in-slice widths
    U[0.5, 1.5], rotation U[0, pi), z width U[0.5, 2.5]), noise 0.04, 16
    uneven blocks of 3..7 slices."""
    shape = (79, 154, 155)
    rp, rn, rb = _seeds(seed)
    xbar = ellipsoid_phantom(shape, 80, rp)
    noise = 0.04 * rn.standard_normal(shape)
    psf = rotated_psf_draws(79, np.random.default_rng(seed + 3), sxy=(0.5, 1.5), sz=(0.5, 2.5))
    return Workload("dense-fp32-155x154x79", shape, xbar, noise, np.zeros(79), np.zeros(79), 5, 11,
                    0.01, 0.02, 0.01, 0.0, uneven_partition(79, 16, 3, 7, rb), grad_rtol=1e-4,
                    extra={"psf": psf})


def tiny_dense(shape, seed, kxy=5, kz=5, nblocks=None, lam=0.01, delta=0.05, eta=0.01, kappa=0.0,
               sxy=(0.5, 1.5), sz=(0.6, 2.0), noise=0.02):
    """Small random problem with rotated per-depth kernels, for tests."""
    w = tiny(shape, seed, kxy=kxy, kz=kz, nblocks=nblocks, lam=lam, delta=delta, eta=eta,
             kappa=kappa, noise=noise)
    w.name = "tiny-dense-%dx%dx%d" % (shape[2], shape[1], shape[0])
    w.extra = {"psf": rotated_psf_draws(shape[0], np.random.default_rng(seed + 3), sxy, sz)}
    return w


def warmstart_train_member(t, seed_base=5_000_000):
    """Training pair t of the learned warm start: a 128x128x32 volume with 25
    ellipsoids (the ellipsoid density of the 256x256x64 volume), the 256x256x64
    workload's PSF law and criterion parameters, 8 uneven blocks of 2..6 slices."""
    base = seed_base + 10 * t
    shape = (32, 128, 128)
    rp, rn, rb = _seeds(base)
    xbar = ellipsoid_phantom(shape, 25, rp)
    noise = 0.02 * rn.standard_normal(shape)
    return Workload("warmstart-train-%d" % t, shape, xbar, noise,
                    linear_schedule(32, 0.5, 3.0), linear_schedule(32, 1.0, 2.0), 7, 7,
                    0.01, 0.02, 0.01, 0.0, uneven_partition(32, 8, 2, 6, rb), grad_rtol=1e-4)


def warmstart_eval_member(e, seed_base=6000):
    """Evaluation volume e of the learned warm start: a fresh draw of the
    256x256x64 workload (same law as plain-fp32-256x256x64, other seeds)."""
    return mid_fp32(seed=seed_base + 10 * e)


def net_layer_shapes(c=16, cin=1):
    """(cout, cin, k) of every layer of the warm-start U-Net, in parameter order."""
    return [(c, cin, 3), (c, c, 3), (2 * c, c, 3), (2 * c, 2 * c, 3), (4 * c, 2 * c, 3),
            (4 * c, 4 * c, 3), (2 * c, 4 * c, 3), (2 * c, 4 * c, 3), (c, 2 * c, 3), (c, 2 * c, 3),
            (1, c, 1)]


def net_init_params(seed, c=16, cin=1, head_scale=0.1, bias=0.0):
    """Seeded starting parameters of the warm-start network (flat float64, the
    parameter layout of the library): weights N(0, 2 / fan_in), the head's
    scaled by head_scale so that x0 starts near y, biases constant."""
    rng = np.random.default_rng(seed)
    out = []
    shapes = net_layer_shapes(c, cin)
    for i, (co, ci, k) in enumerate(shapes):
        fan = ci * k ** 3
        w = rng.standard_normal(co * ci * k ** 3) * np.sqrt(2.0 / fan)
        if i == len(shapes) - 1:
            w *= head_scale
        out.append(w)
        out.append(np.full(co, bias))
    return np.concatenate(out)


WORKLOADS = {
    "plain-fp64-64x64x16": small_plain_fp64,
    "plain-fp32-256x256x64": mid_fp32,
    "plain-fp32-512x512x128": large_fp32,
    "dense-fp32-256x256x24": dense_fp32_256x256x24,
    "dense-fp32-155x154x79": dense_fp32_155x154x79,
}
