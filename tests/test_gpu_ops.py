"""GPU parity of the operators behind the C interface: H, H^T and grad f
against the FP64 oracle, element by element, on shapes that span several
tiles with ragged tails, and the GPU adjoint identity.

Tolerances: FP64 -- every output is a sum of at most K_z + K_x + K_y
rounded products in a different order than the oracle's, so the difference is
bounded by a few dozen ulps of the largest |term| sum; 1e-13 of the output's
max. FP32 -- inputs are identical (rounded once), the stencil arithmetic is
float: about (K_z + K_x + K_y) * 2^-24 relative to the sum of |terms|; 2e-6 of
the max for H and H^T, and for grad f (whose TV part divides by the local
gradient magnitude, amplifying rounding up to 1/delta) 5e-5.
"""
import numpy as np
import pytest

from paper_2002_02328_amd import binding
from gpu_common import pair, maxrel

pytestmark = pytest.mark.gpu

SHAPES = [(5, 37, 150), (3, 16, 64), (4, 5, 7), (1, 20, 70), (9, 33, 65)]
KERNELS = [(3, 3, 3), (5, 5, 5), (7, 7, 7), (9, 9, 9), (9, 3, 5), (1, 1, 1), (3, 5, 1)]


def cases():
    out = []
    for si, shape in enumerate(SHAPES):
        for ki, ks in enumerate(KERNELS):
            if (si + ki) % 2 == 0 or shape == (5, 37, 150):
                out.append((shape, ks))
    return out


@pytest.mark.parametrize("shape,ks", cases())
@pytest.mark.parametrize("prec,rows", [(binding.FP64, 16), (binding.FP32, 16), (binding.FP32, 32)])
def test_H_HT_parity(orc, shape, ks, prec, rows):
    g, o, y = pair(orc, shape, prec, seed=sum(shape) + sum(ks), kx=ks[0], ky=ks[1], kz=ks[2],
                   tables="asym")
    g.set_option(binding.OPT_TILE_ROWS_AUX, rows)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(shape)
    if prec == binding.FP32:
        v = v.astype(np.float32).astype(np.float64)
    tol = 1e-13 if prec == binding.FP64 else 2e-6
    h_gpu, h_ref = g.H(v), o.H(v)
    assert maxrel(h_gpu, h_ref) <= tol
    t_gpu, t_ref = g.HT(v), o.HT(v)
    assert maxrel(t_gpu, t_ref) <= tol


@pytest.mark.parametrize("shape,ks", cases()[:6])
@pytest.mark.parametrize("prec,rows", [(binding.FP64, 16), (binding.FP32, 16), (binding.FP32, 32)])
@pytest.mark.parametrize("kappa", [0.0, 0.05])
def test_grad_parity(orc, shape, ks, prec, rows, kappa):
    g, o, y = pair(orc, shape, prec, seed=3 + sum(shape), kx=ks[0], ky=ks[1], kz=ks[2],
                   lam=0.02, delta=0.05, eta=0.5, kappa=kappa)
    g.set_option(binding.OPT_TILE_ROWS_UPDATE, rows)
    rng = np.random.default_rng(11)
    x = rng.uniform(-0.2, 1.2, size=shape)
    if prec == binding.FP32:
        x = x.astype(np.float32).astype(np.float64)
    tol = 1e-12 if prec == binding.FP64 else 5e-5
    assert maxrel(g.grad(x), o.grad(x)) <= tol


@pytest.mark.parametrize("prec", [binding.FP64, binding.FP32])
def test_gpu_adjoint_identity(orc, prec):
    shape = (11, 45, 131)
    g, o, y = pair(orc, shape, prec, seed=5, kx=7, ky=5, kz=9, tables="asym")
    rng = np.random.default_rng(5)
    a = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    ha = g.H(a).astype(np.float64)
    htb = g.HT(b).astype(np.float64)
    a64 = a.astype(g.dtype).astype(np.float64)
    b64 = b.astype(g.dtype).astype(np.float64)
    lhs, rhs = float((ha * b64).sum()), float((a64 * htb).sum())
    tol = 1e-13 if prec == binding.FP64 else 1e-5
    assert abs(lhs - rhs) <= tol * np.linalg.norm(ha) * np.linalg.norm(b64)


def test_eval_matches_oracle(orc):
    shape = (6, 40, 90)
    g, o, y = pair(orc, shape, binding.FP64, seed=9, lam=0.03, delta=0.02, eta=0.4, kappa=0.1,
                   nslices=[2, 4])
    rng = np.random.default_rng(3)
    x = rng.uniform(-0.3, 1.3, size=shape)
    g.set_x0(x)
    f, gn = g.eval()
    assert abs(f - o.f(x)) <= 1e-12 * abs(o.f(x))
    assert abs(gn - o.grad_norm(x)) <= 1e-11 * o.grad_norm(x)
