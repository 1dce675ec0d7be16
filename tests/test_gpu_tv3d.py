"""GPU parity of the total variation taken over the volume (bd3mg_set_tv3d:
V^Z inside the root next to V^X and V^Y) against the FP64 oracle with the
same option: the gradient element by element, f and ||grad f||, single block
steps (the 2x2 system, whose z-difference products now carry the weight
2 kappa + lambda omega and reach the slice below the block), whole
trajectories in the coloured, sequential and asynchronous-round schedules,
the general (dense) PSF, the colouring gap without z blur, the Lipschitz
bound, and the refusals.

Tolerances are those of the slice-TV tests of the same operations: FP64
gradient 1e-12 of the max (rounding order only), FP32 5e-5 (the TV weight
amplifies rounding by up to 1/delta); FP64 trajectories 1e-10 relative in x
after a few dozen sweeps (the GPU updates the residual incrementally, the
oracle recomputes it: rounding carried along by the iteration).
"""
import numpy as np
import pytest

import oracle
from paper_2002_02328_amd import binding, inputs
from gpu_common import pair, rel, maxrel, rounded

pytestmark = pytest.mark.gpu

SHAPES = [((6, 37, 150), (5, 5, 5)), ((5, 16, 64), (3, 3, 3)), ((4, 5, 7), (3, 5, 1)),
          ((9, 33, 65), (7, 7, 7)), ((2, 20, 70), (1, 1, 1))]


@pytest.mark.parametrize("shape,ks", SHAPES)
@pytest.mark.parametrize("prec", [binding.FP64, binding.FP32])
@pytest.mark.parametrize("kappa", [0.0, 0.05])
def test_grad_parity(orc, shape, ks, prec, kappa):
    g, o, y = pair(orc, shape, prec, seed=3 + sum(shape), kx=ks[0], ky=ks[1], kz=ks[2],
                   lam=0.02, delta=0.05, eta=0.5, kappa=kappa, tv3d=True)
    rng = np.random.default_rng(11)
    x = rounded(rng.uniform(-0.2, 1.2, size=shape), prec)
    tol = 1e-12 if prec == binding.FP64 else 5e-5
    ref = o.grad(x)
    assert maxrel(g.grad(x), ref) <= tol
    # the z part is really there: the slice-TV gradient differs by far more
    o2 = orc.Problem(y, o.gx, o.gy, o.gz, lam=0.02, delta=0.05, eta=0.5, kappa=kappa)
    if shape[0] > 1:
        assert maxrel(o2.grad(x), ref) > 100 * tol


def test_eval_matches_oracle(orc):
    shape = (6, 40, 90)
    g, o, y = pair(orc, shape, binding.FP64, seed=9, lam=0.03, delta=0.02, eta=0.4, kappa=0.1,
                   nslices=[2, 4], tv3d=True)
    x = np.random.default_rng(3).uniform(-0.3, 1.3, size=shape)
    g.set_x0(x)
    f, gn = g.eval()
    assert abs(f - o.f(x)) <= 1e-12 * abs(o.f(x))
    assert abs(gn - o.grad_norm(x)) <= 1e-11 * o.grad_norm(x)


@pytest.mark.parametrize("kz,kappa", [(3, 0.0), (1, 0.0), (5, 0.04)])
def test_block_steps_match_oracle(orc, kz, kappa):
    shape = (10, 37, 70)
    nsl = [3, 2, 4, 1]
    g, o, y = pair(orc, shape, binding.FP64, seed=2, kx=5, ky=5, kz=kz, lam=0.02, delta=0.03,
                   eta=0.3, kappa=kappa, nslices=nsl, tv3d=True)
    g.set_x0(None)
    x = y.copy()
    d = np.zeros(shape)
    z0 = np.concatenate([[0], np.cumsum(nsl)[:-1]])
    for b in [0, 2, 1, 3, 0, 2, 3, 1, 0]:  # second visits exercise the memory term
        info_g = g.block_step(b)
        info_o = o.block_step(x, d, int(z0[b]), nsl[b])
        assert np.allclose(info_g, info_o, rtol=1e-10, atol=1e-300), (b, info_g, info_o)
        assert rel(g.get_x(), x) <= 1e-12
        assert rel(g.get_dprev(), d) <= 1e-10


@pytest.mark.parametrize("schedule", [binding.SCHED_COLORED, binding.SCHED_SEQUENTIAL])
@pytest.mark.parametrize("shape,nsl,kz", [((12, 40, 90), [3, 2, 4, 3], 5), ((8, 24, 70), [1] * 8, 1),
                                          ((9, 19, 33), [2, 3, 1, 3], 3)])
def test_trajectory_fp64(orc, schedule, shape, nsl, kz):
    g, o, y = pair(orc, shape, binding.FP64, seed=sum(nsl) + kz, kx=5, ky=3, kz=kz, lam=0.02,
                   delta=0.03, eta=0.3, nslices=nsl, schedule=schedule, tv3d=True)
    nc, order, color = g.get_schedule()
    g.set_x0(None)
    x, d = y.copy(), np.zeros(shape)
    f_prev = o.f(x)
    done = 0
    for cp in (1, 5, 25):
        res = g.run(cp - done)
        o.run(x, d, nsl, order, cp - done, history=False)
        done = cp
        assert rel(g.get_x(), x) <= 1e-10, cp
        fo = o.f(x)
        assert abs(res["f"] - fo) <= 1e-12 * abs(fo), cp
        assert fo < f_prev
        f_prev = fo


def test_colouring_gap_without_z_blur(orc):
    """With kz = 1 blocks interact only through the z difference of the TV:
    neighbours take different colours (gap 1), every other block shares one."""
    nsl = [2, 1, 3, 1, 1, 2]
    g, o, y = pair(orc, (10, 8, 8), binding.FP64, seed=1, kx=3, ky=3, kz=1, nslices=nsl, tv3d=True)
    nc, order, color = g.get_schedule()
    onc, oorder, ocolor = orc.color_schedule(nsl, 1)
    assert nc == onc == 2
    assert np.array_equal(order, oorder) and np.array_equal(color, ocolor)
    g.set_tv3d(False)
    assert g.get_schedule()[0] == 1


def test_round_trajectory_with_inflation(orc):
    nsl = [2, 3, 2, 3]
    g, o, y = pair(orc, (10, 30, 50), binding.FP64, seed=4, kx=5, ky=5, kz=5, lam=0.02, delta=0.03,
                   eta=0.3, nslices=nsl, schedule=binding.SCHED_ROUND, mu=0.5, tv3d=True)
    g.set_x0(None)
    x, d = y.copy(), np.zeros(y.shape)
    res = g.run(8)
    o.run_round(x, d, nsl, 8, history=False)
    assert rel(g.get_x(), x) <= 1e-10
    assert abs(res["f"] - o.f(x)) <= 1e-12 * abs(o.f(x))


def test_dense_psf_trajectory(orc):
    shape, nsl = (9, 24, 70), [2, 3, 1, 3]
    nz, ny, nx = shape
    rng = np.random.default_rng(8)
    pk = oracle.rotated_gauss_kernels(rng.uniform(0.5, 2.0, nz), rng.uniform(0.5, 2.0, nz),
                                      rng.uniform(0, np.pi, nz), rng.uniform(0.6, 3.0, nz), 5, 5)
    w = inputs.tiny(shape, 8)
    y = oracle.Problem.with_kernels(np.zeros(shape), pk).H(w.xbar) + w.noise
    o = oracle.Problem.with_kernels(y, pk, lam=0.02, delta=0.03, eta=0.3, kappa=0.01, tv3d=True)
    g = binding.Problem(nx, ny, nz, binding.FP64)
    g.set_psf_dense(pk)
    g.set_params(0.02, 0.03, 0.3, 0.01)
    g.set_tv3d(True)
    g.set_data(y)
    g.set_blocks(np.asarray(nsl, np.int32))
    nc, order, color = g.get_schedule()
    g.set_x0(None)
    x, d = y.copy(), np.zeros(shape)
    g.run(10)
    o.run(x, d, nsl, order, 10, history=False)
    assert rel(g.get_x(), x) <= 1e-10
    assert rel(g.get_dprev(), d) <= 1e-9


def test_fp32_tracks_fp64_oracle(orc):
    shape, nsl = (12, 48, 96), [3, 3, 3, 3]
    g, o, y = pair(orc, shape, binding.FP32, seed=6, kx=5, ky=5, kz=5, lam=0.02, delta=0.03,
                   eta=0.3, nslices=nsl, tv3d=True)
    nc, order, color = g.get_schedule()
    g.set_x0(None)
    x, d = y.copy(), np.zeros(shape)
    res = g.run(30)
    o.run(x, d, nsl, order, 30, history=False)
    assert rel(g.get_x(), x) <= 1e-4
    assert abs(res["f"] - o.f(x)) <= 1e-5 * abs(o.f(x))


def test_lipschitz_bound_and_refusals(orc):
    g, o, y = pair(orc, (6, 16, 24), binding.FP64, seed=5, lam=0.3, delta=0.05, nslices=[3, 3], tv3d=True)
    L = g.lipschitz_bound()
    assert abs(L - o.lipschitz_bound()) <= 1e-14 * L
    g.set_tv3d(False)
    assert abs(L - g.lipschitz_bound() - 4 * 0.3 / 0.05) <= 1e-12 * L
    with pytest.raises(binding.Bd3mgError):
        g.set_tv3d(2)
    g.set_tv3d(True)
    with pytest.raises(binding.Bd3mgError):
        g.set_method(binding.METHOD_ASYNC_MM, n_inner=3)
    g.set_tv3d(False)
    g.set_method(binding.METHOD_ASYNC_MM, n_inner=3)
    with pytest.raises(binding.Bd3mgError):
        g.set_tv3d(True)
