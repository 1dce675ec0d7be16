"""Shared set-up of GPU parity tests: the same seeded inputs go to the HIP
library (through the C interface) and to the FP64 oracle."""
import numpy as np

from paper_2002_02328_amd import binding, inputs


def rounded(a, prec):
    """Inputs are rounded once to the storage precision; both sides use them."""
    if prec == binding.FP32:
        return np.asarray(a, dtype=np.float32).astype(np.float64)
    return np.asarray(a, dtype=np.float64)


def pair(orc, shape, prec, seed, kx=5, ky=5, kz=5, tables="gauss", lam=0.01, delta=0.02, eta=0.01,
         kappa=0.0, nslices=None, schedule=binding.SCHED_COLORED, y=None, mu=0.0, tv3d=False):
    """(gpu problem, oracle problem, y) with identical rounded inputs (mu: the
    curvature inflation of both; tv3d: the total variation along z too)."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    if tables == "gauss":
        gx = orc.gauss_table(np.linspace(0.5, 2.0, nz), kx)
        gy = orc.gauss_table(np.linspace(0.7, 1.6, nz), ky)
        gz = orc.gauss_table(np.linspace(1.0, 2.0, nz), kz)
    else:  # asymmetric, non-normalised: exposes transposes and index mistakes
        gx = rng.uniform(0.05, 0.4, size=(nz, kx))
        gy = rng.uniform(0.05, 0.4, size=(nz, ky))
        gz = rng.uniform(0.05, 0.4, size=(nz, kz))
    gx, gy, gz = rounded(gx, prec), rounded(gy, prec), rounded(gz, prec)
    if y is None:
        w = inputs.tiny(shape, seed, kxy=kx, kz=kz)
        p0 = orc.Problem(np.zeros(shape), gx, gy, gz)
        y = p0.H(w.xbar) + w.noise
    y = rounded(y, prec)
    o = orc.Problem(y, gx, gy, gz, lam=lam, delta=delta, eta=eta, kappa=kappa, mu=mu, tv3d=tv3d)
    g = binding.Problem(nx, ny, nz, prec)
    if mu:
        g.set_inflation(mu)
    if tv3d:
        g.set_tv3d(True)
    g.set_psf_separable(gx, gy, gz)
    g.set_params(lam, delta, eta, kappa)
    g.set_data(y)
    if nslices is not None:
        g.set_blocks(nslices, schedule)
    return g, o, y


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def maxrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
