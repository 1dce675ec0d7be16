"""Element-wise FP32 parity of the single-precision kernel instances (the
32-row direction and update tiles exist in FP32 only) against the FP64
oracle, on shapes whose rows and columns leave ragged tiles (ny not a
multiple of 16 or 32, nx not a multiple of 64), at both tile heights.

Block steps.  Before each step the oracle is given the GPU's current x and
previous steps (FP32 values), so each step's rounding is compared on its
own (the GPU's maintained residual still carries the drift of the earlier
steps).  Tolerances follow the arithmetic: an FP32 stencil output with
M = kx + ky + kz rounded terms has relative error at most about M 2^-24 of
its sum of |terms| (the tables are non-negative), so a curvature or
gradient inner product of such outputs, accumulated in FP64, is within
tol_B = 4 M 2^-24 relative; the 2x2 solve multiplies that by the
condition number of B (rank-one branch: by 2); x is stored in FP32
(2^-24 |x| per element) and moves by the step, whose error is tol_u of
its size; the previous step is tol_u of its size plus its own rounding.
A dropped term, a sign, the wrong slice's kernel or a transposed operand
changes B, c or u by 1e-2 or more.

Trajectories.  A few sweeps from x0 = y, GPU (FP32) against oracle (FP64)
on the same rounded inputs: each step differs by the per-step errors above
and the iteration carries them along; the bound is 2^-24 |x| plus 4 M 2^-24
of the distance travelled, max|x - y|.
"""
import numpy as np
import pytest

from paper_2002_02328_amd import binding
from gpu_common import pair

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -24
SHAPES = [((10, 37, 70), (5, 5, 3), [3, 2, 4, 1]),
          ((12, 45, 130), (7, 7, 7), [2, 4, 3, 3]),
          ((9, 20, 67), (9, 3, 5), [4, 1, 4])]


def _fp32(orc, shape, ks, nsl, rows, seed):
    g, o, y = pair(orc, shape, binding.FP32, seed=seed, kx=ks[0], ky=ks[1], kz=ks[2],
                   lam=0.02, delta=0.03, eta=0.3, nslices=nsl)
    for opt in (binding.OPT_TILE_ROWS_DIRS, binding.OPT_TILE_ROWS_UPDATE, binding.OPT_TILE_ROWS_AUX):
        g.set_option(opt, rows)
    return g, o, y


@pytest.mark.parametrize("rows", [16, 32])
@pytest.mark.parametrize("shape,ks,nsl", SHAPES)
def test_fp32_block_steps_match_oracle(orc, shape, ks, nsl, rows):
    g, o, y = _fp32(orc, shape, ks, nsl, rows, seed=2 + sum(shape))
    g.set_x0(None)
    M = sum(ks)
    tol_B = 4 * M * EPS
    z0 = np.concatenate([[0], np.cumsum(nsl)[:-1]])
    nb = len(nsl)
    for b in [0, 2, 1, 3 % nb, 0, 2, 3 % nb, 1, 0]:  # second visits exercise the memory term
        x = g.get_x().astype(np.float64)
        d = g.get_dprev().astype(np.float64)
        xin = x.copy()
        io = np.asarray(o.block_step(x, d, int(z0[b]), nsl[b]))
        ig = np.asarray(g.block_step(b))
        b11, b12, b22 = io[:3]
        rank1 = b11 * b22 - b12 * b12 <= 1e-12 * b11 * b22
        tol_u = 2 * tol_B if rank1 else tol_B * np.linalg.cond(np.array([[b11, b12], [b12, b22]]))
        where = (shape, rows, b)
        assert np.max(np.abs(ig[:3] - io[:3])) <= tol_B * np.max(np.abs(io[:3])), (where, ig, io)
        assert np.max(np.abs(ig[3:5] - io[3:5])) <= tol_B * np.max(np.abs(io[3:5])), (where, ig, io)
        assert np.max(np.abs(ig[5:7] - io[5:7])) <= tol_u * np.max(np.abs(io[5:7])), (where, ig, io)
        assert abs(ig[7] - io[7]) <= tol_B * io[7], (where, ig, io)
        step = np.max(np.abs(x - xin))
        assert np.max(np.abs(g.get_x() - x)) <= 2 * EPS * np.max(np.abs(x)) + tol_u * step, where
        assert np.max(np.abs(g.get_dprev() - d)) <= (2 * EPS + tol_u) * np.max(np.abs(d)), where
    g.close()


@pytest.mark.parametrize("rows", [16, 32])
@pytest.mark.parametrize("shape,ks,nsl,sweeps", [((12, 45, 130), (7, 7, 7), [2, 4, 3, 3], 5),
                                                 ((16, 37, 70), (5, 5, 5), [3, 2, 4, 1, 6], 30)])
def test_fp32_trajectory_max_norm(orc, shape, ks, nsl, sweeps, rows):
    g, o, y = _fp32(orc, shape, ks, nsl, rows, seed=5 + sum(shape))
    nc, order, _ = g.get_schedule()
    g.set_x0(None)
    g.run(sweeps, check_every=0)
    x = y.copy()
    d = np.zeros(shape)
    o.run(x, d, nsl, order, sweeps, history=False)
    err = np.max(np.abs(g.get_x() - x))
    bound = 2 * EPS * np.max(np.abs(x)) + 4 * sum(ks) * EPS * np.max(np.abs(x - y))
    print("FP32 %s, %d-row tiles, %d sweeps: max|x_gpu - x_oracle| = %.3e (bound %.3e)"
          % (shape, rows, sweeps, err, bound))
    assert err <= bound
    dg = g.get_dprev()
    assert np.max(np.abs(dg - d)) <= 2 * EPS * np.max(np.abs(x)) + 4 * sum(ks) * EPS * np.max(np.abs(x - y))
    g.close()
