"""GPU parity of the general per-depth PSF (the rotated Gaussian kernels of
random variance and rotation the paper's experiments use, Sec. 3.1): the
operators H, H^T and grad f, the objective, block steps, coloured and round
trajectories and batches, against the FP64 oracle's general-kernel path.

Tolerances: FP64 within 1e-12 for the operators (summation order only) and
1e-9 for trajectories (as for the separable PSF); FP32 within 1e-5 for the
operators (a sum of up to 11 x 11 x 21 products in single precision) and 2e-4
for trajectories.
"""
import numpy as np
import pytest

import oracle
from paper_2002_02328_amd import binding, inputs
from gpu_common import rel, rounded

pytestmark = pytest.mark.gpu


def kernels(nz, kx, ky, kz, seed, kind="gauss"):
    rng = np.random.default_rng(seed)
    if kind == "gauss":
        k = max(kx, ky)
        pk = oracle.rotated_gauss_kernels(rng.uniform(0.5, 2.0, nz), rng.uniform(0.5, 2.0, nz),
                                          rng.uniform(0, np.pi, nz), rng.uniform(0.6, 3.0, nz), k, kz)
        b0, a0 = (k - ky) // 2, (k - kx) // 2
        return pk[:, :, b0:b0 + ky, a0:a0 + kx].copy()
    # asymmetric, depth-variant, not normalised: exposes transposes and index mistakes
    return rng.uniform(0.01, 0.2, (nz, kz, ky, kx))


def setup(shape, prec, kx, ky, kz, seed=3, kind="gauss", nslices=None, schedule=binding.SCHED_COLORED,
          lam=0.01, delta=0.05, eta=0.01, kappa=0.0, mu=0.0):
    nz, ny, nx = shape
    pk = rounded(kernels(nz, kx, ky, kz, seed, kind), prec)
    w = inputs.tiny(shape, seed)
    y = rounded(oracle.Problem.with_kernels(np.zeros(shape), pk).H(w.xbar) + w.noise, prec)
    o = oracle.Problem.with_kernels(y, pk, lam=lam, delta=delta, eta=eta, kappa=kappa, mu=mu)
    g = binding.Problem(nx, ny, nz, prec)
    g.set_psf_dense(pk)
    g.set_params(lam, delta, eta, kappa)
    g.set_inflation(mu)
    g.set_data(y)
    if nslices is not None:
        g.set_blocks(np.asarray(nslices, np.int32), schedule)
    return g, o, y


OPS = [((9, 40, 70), 5, 5, 5, "gauss"), ((7, 33, 65), 3, 7, 9, "asym"), ((12, 70, 130), 11, 11, 21, "gauss"),
       ((5, 21, 19), 11, 9, 3, "asym"), ((1, 64, 64), 5, 5, 1, "asym"), ((6, 30, 40), 1, 1, 5, "asym")]


@pytest.mark.parametrize("prec,tol", [(binding.FP64, 1e-12), (binding.FP32, 1e-5)])
@pytest.mark.parametrize("shape,kx,ky,kz,kind", OPS)
def test_operators_match_oracle(orc, prec, tol, shape, kx, ky, kz, kind):
    g, o, y = setup(shape, prec, kx, ky, kz, kind=kind)
    v = rounded(np.random.default_rng(4).random(shape), prec)
    assert rel(g.apply(binding.OP_H, v), o.H(v)) <= tol
    assert rel(g.apply(binding.OP_HT, v), o.HT(v)) <= tol
    assert rel(g.apply(binding.OP_GRAD, v), o.grad(v)) <= 10 * tol


def test_objective_and_lipschitz_bound(orc):
    g, o, y = setup((8, 37, 66), binding.FP64, 7, 5, 9, nslices=[2, 3, 3], kappa=0.02)
    g.set_x0(None)
    f, gn = g.eval()
    assert abs(f - o.f(y)) <= 1e-12 * abs(o.f(y))
    assert abs(gn - o.grad_norm(y)) <= 1e-11 * o.grad_norm(y)
    assert abs(g.lipschitz_bound() - o.lipschitz_bound()) <= 1e-14 * o.lipschitz_bound()


@pytest.mark.parametrize("shape,nslices,kxy,kz,kappa", [
    ((9, 24, 70), [2, 3, 1, 3], 5, 5, 0.0),
    ((10, 33, 40), [4, 2, 4], 11, 21, 0.03),
    ((6, 20, 30), [1, 1, 2, 1, 1], 3, 7, 0.0),
])
def test_coloured_trajectory_fp64(orc, shape, nslices, kxy, kz, kappa):
    g, o, y = setup(shape, binding.FP64, kxy, kxy, kz, nslices=nslices, kappa=kappa)
    nc, order, color = g.get_schedule()
    g.set_x0(None)
    x, d = y.copy(), np.zeros(shape)
    done = 0
    for cp in (1, 4, 12):
        g.run(cp - done)
        o.run(x, d, nslices, order, cp - done, history=False)
        done = cp
        assert rel(g.get_x(), x) <= 1e-9, cp
        assert rel(g.get_dprev(), d) <= 1e-8, cp


def test_round_trajectory_and_block_step_fp64(orc):
    nslices = [2, 2, 3, 1]
    g, o, y = setup((8, 30, 50), binding.FP64, 5, 5, 7, nslices=nslices, schedule=binding.SCHED_ROUND, mu=0.4)
    g.set_x0(None)
    x, d = y.copy(), np.zeros(y.shape)
    g.run(6)
    o.run_round(x, d, nslices, 6, history=False)
    assert rel(g.get_x(), x) <= 1e-9
    # one block alone (block 2: slices 4..6), from the current state
    info = g.block_step(2)
    oi = o.block_step(x, d, 4, 3)
    assert np.allclose(info, oi, rtol=1e-9, atol=1e-14)
    assert rel(g.get_x(), x) <= 1e-9


def test_fp32_tracks_fp64_oracle(orc):
    nslices = [3, 2, 4, 3]
    g, o, y = setup((12, 48, 80), binding.FP32, 11, 11, 21, nslices=nslices)
    nc, order, color = g.get_schedule()
    g.set_x0(None)
    g.run(15)
    x, d = y.copy(), np.zeros(y.shape)
    o.run(x, d, nslices, order, 15, history=False)
    assert rel(g.get_x(), x) <= 2e-4


def test_stop_rule_matches_oracle(orc):
    nslices = [2, 2, 2, 2]
    g, o, y = setup((8, 16, 24), binding.FP64, 5, 5, 5, nslices=nslices)
    nc, order, color = g.get_schedule()
    g.set_x0(None)
    res = g.run(400, grad_rtol=1e-4, check_every=1)
    x, d = y.copy(), np.zeros(y.shape)
    s, fh, gh = o.run(x, d, nslices, order, 400, grad_rtol=1e-4)
    assert res["converged"] == 1 and res["sweeps"] == s


def test_batch_equals_single_runs(orc):
    cases = [((9, 24, 70), [2, 3, 1, 3], 5, 5), ((10, 33, 40), [4, 2, 4], 11, 21)]
    single = []
    for i, (shape, ns, kxy, kz) in enumerate(cases):
        g, o, y = setup(shape, binding.FP32, kxy, kxy, kz, seed=20 + i, nslices=ns)
        g.set_x0(None)
        g.run(6, check_every=0)
        single.append(g.get_x())
    probs = []
    for i, (shape, ns, kxy, kz) in enumerate(cases):
        g = setup(shape, binding.FP32, kxy, kxy, kz, seed=20 + i, nslices=ns)[0]
        g.set_x0(None)
        probs.append(g)
    b = binding.Batch(probs)
    b.run(6)
    for g, xs in zip(probs, single):
        assert np.array_equal(g.get_x(), xs)


def test_full_size_rotated_workload_one_sweep_against_oracle(orc):
    """The 256x256x24 workload (kernels 11x11x21): one FP32 sweep against the
    FP64 oracle's sweep from the same rounded inputs."""
    w = inputs.dense_fp32_256x256x24()
    ps = w.extra["psf"]
    pk = rounded(oracle.rotated_gauss_kernels(ps["sx"], ps["sy"], ps["theta"], ps["sz"], w.kxy, w.kz),
                 binding.FP32)
    y = rounded(oracle.Problem.with_kernels(np.zeros(w.shape), pk).H(w.xbar) + w.noise, binding.FP32)
    o = oracle.Problem.with_kernels(y, pk, lam=w.lam, delta=w.delta, eta=w.eta)
    nz, ny, nx = w.shape
    g = binding.Problem(nx, ny, nz, binding.FP32)
    g.set_psf_dense(pk)
    g.set_params(w.lam, w.delta, w.eta, w.kappa)
    g.set_data(y.astype(np.float32))
    g.set_blocks(w.nslices, binding.SCHED_COLORED)
    nc, order, color = g.get_schedule()
    g.set_x0(None)
    g.run(1)
    x, d = y.copy(), np.zeros(y.shape)
    o.run(x, d, w.nslices, order, 1, history=False)
    assert rel(g.get_x(), x) <= 1e-5


def test_set_psf_dense_rejects_bad_kernels(orc):
    g = binding.Problem(20, 16, 6, binding.FP32)
    ok = np.full((6, 3, 3, 3), 1.0 / 27)
    g.set_psf_dense(ok)
    for bad in (np.ones((6, 3, 4, 3)), np.ones((6, 3, 3, 13)), np.ones((6, 23, 3, 3)), np.ones((6, 2, 3, 3))):
        with pytest.raises(binding.Bd3mgError) as e:
            g.set_psf_dense(bad)
        assert e.value.status == binding.ERR_ARG
    nan = ok.copy()
    nan[2, 1, 1, 1] = np.nan
    with pytest.raises(binding.Bd3mgError):
        g.set_psf_dense(nan)
    with pytest.raises(ValueError):
        g.set_psf_dense(np.ones((5, 3, 3, 3)))
    g.close()


def test_switching_between_separable_and_general_psf(orc):
    """A separable PSF given as general kernels (tensor products) and as
    factors gives the same trajectory, and switching back and forth works."""
    shape, nslices = (8, 30, 70), [3, 2, 3]
    nz, ny, nx = shape
    rng = np.random.default_rng(40)
    gx, gy, gz = (oracle.gauss_table(rng.uniform(0.6, 1.8, nz), k) for k in (5, 5, 3))
    pk = np.einsum("kc,kb,ka->kcba", gz, gy, gx)
    w = inputs.tiny(shape, 41)
    y = oracle.Problem(np.zeros(shape), gx, gy, gz).H(w.xbar) + w.noise
    g = binding.Problem(nx, ny, nz, binding.FP64)
    g.set_params(0.01, 0.05, 0.01)
    g.set_data(y)
    g.set_psf_separable(gx, gy, gz)
    g.set_blocks(nslices)
    g.set_x0(None)
    g.run(5)
    xs = g.get_x()
    g.set_psf_dense(pk)
    g.set_x0(None)
    g.run(5)
    xd = g.get_x()
    assert rel(xd, xs) <= 1e-12
    g.set_psf_separable(gx, gy, gz)
    g.set_x0(None)
    g.run(5)
    assert np.array_equal(g.get_x(), xs)
    g.close()
