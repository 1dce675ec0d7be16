"""GPU parity of batched BD3MG: many problems of uneven sizes advanced together
through one graph launch per two sweeps.

The batch runs the same kernels with the same arguments as single-problem
runs, the direction pass of each problem blurring d1 only or both directions
on the same sweeps as its single run (by its own sweep count), so a batched
run must equal the single runs bitwise, with H dp kept (the default) and
without (BD3MG_OPT_HDP_EVERY = 0); against the FP64 oracle the usual FP64 /
FP32 bounds apply (see test_gpu_solver).
"""
import numpy as np
import pytest

from paper_2002_02328_amd import binding, inputs
from gpu_common import rel, rounded

pytestmark = pytest.mark.gpu


def setup(orc, w, prec, hdp_every=None):
    gxy = rounded(orc.gauss_table(w.sigma_xy, w.kxy), prec)
    gz = rounded(orc.gauss_table(w.sigma_z, w.kz), prec)
    y = rounded(orc.Problem(np.zeros(w.shape), gxy, gxy, gz).H(w.xbar) + w.noise, prec)
    nz, ny, nx = w.shape
    g = binding.Problem(nx, ny, nz, prec)
    g.set_psf_separable(gxy, gxy, gz)
    g.set_params(w.lam, w.delta, w.eta, w.kappa)
    g.set_data(y)
    g.set_blocks(w.nslices)
    g.set_x0(None)
    if hdp_every is not None:
        g.set_option(binding.OPT_HDP_EVERY, hdp_every)
    o = orc.Problem(y, gxy, gxy, gz, lam=w.lam, delta=w.delta, eta=w.eta, kappa=w.kappa)
    return g, o, y


def small_members():
    return [inputs.tiny((9, 40, 70), 31, kxy=5, kz=5, nblocks=3),
            inputs.tiny((6, 70, 33), 32, kxy=3, kz=3, nblocks=2),
            inputs.tiny((12, 17, 130), 33, kxy=7, kz=5, nblocks=4),
            inputs.tiny((5, 64, 64), 34, kxy=9, kz=1, nblocks=5)]


@pytest.mark.parametrize("hdp_every", [None, 0])
@pytest.mark.parametrize("sweeps", [6, 7, 70])
def test_batch_equals_single_runs_bitwise(orc, sweeps, hdp_every):
    ws = small_members()
    single = []
    for w in ws:
        g, o, y = setup(orc, w, binding.FP32, hdp_every)
        g.run(sweeps, check_every=0)
        single.append(g.get_x())
    probs = [setup(orc, w, binding.FP32, hdp_every)[0] for w in ws]
    b = binding.Batch(probs)
    res = b.run(sweeps)
    for g, xs, r in zip(probs, single, res):
        assert r["sweeps"] == sweeps
        assert np.array_equal(g.get_x(), xs)
    # a second run continues from the state, as single runs do
    b.run(2)
    assert all(g.get_state()[3] == sweeps + 2 for g in probs)


def fusable_members():
    """Problems of different shapes and partitions with one kernel shape
    (PSF 5x5x5), so that one fused launch per pass serves them all."""
    return [inputs.tiny((9, 40, 70), 41, kxy=5, kz=5, nblocks=3),
            inputs.tiny((6, 70, 33), 42, kxy=5, kz=5, nblocks=2),
            inputs.tiny((12, 17, 130), 43, kxy=5, kz=5, nblocks=4),
            inputs.tiny((5, 64, 64), 44, kxy=5, kz=5, nblocks=5),
            inputs.tiny((16, 23, 91), 45, kxy=5, kz=5, nblocks=7)]


@pytest.mark.parametrize("prec,hdp_every", [(binding.FP32, None), (binding.FP64, None), (binding.FP32, 0)])
@pytest.mark.parametrize("sweeps", [6, 7, 70])
def test_fused_batch_equals_single_runs_bitwise(orc, prec, sweeps, hdp_every):
    ws = fusable_members()
    single = []
    for w in ws:
        g, o, y = setup(orc, w, prec, hdp_every)
        g.run(sweeps, check_every=0)
        single.append((g.get_x(), g.get_dprev()))
    probs = [setup(orc, w, prec, hdp_every)[0] for w in ws]
    b = binding.Batch(probs)
    assert b.set_mode(binding.BATCH_FUSED)
    res = b.run(sweeps)
    for g, (xs, ds), r in zip(probs, single, res):
        assert r["sweeps"] == sweeps
        assert np.array_equal(g.get_x(), xs) and np.array_equal(g.get_dprev(), ds)
    # and the branch mode gives the same again
    probs2 = [setup(orc, w, prec, hdp_every)[0] for w in ws]
    b2 = binding.Batch(probs2)
    assert not b2.set_mode(binding.BATCH_BRANCHES)
    b2.run(sweeps)
    for g, g2 in zip(probs, probs2):
        assert np.array_equal(g.get_x(), g2.get_x())


def test_fused_batch_with_a_tolerance_and_fallback(orc):
    ws = fusable_members()[:3]
    made = [setup(orc, w, binding.FP64) for w in ws]
    b = binding.Batch([m[0] for m in made])
    assert b.set_mode(binding.BATCH_FUSED)
    res = b.run(400, grad_rtol=1e-3, check_every=4)
    for (g, o, y), w, r in zip(made, ws, res):
        assert r["converged"] == 1 and r["sweeps"] % 4 == 0
        g2 = setup(orc, w, binding.FP64)[0]
        g2.run(r["sweeps"], check_every=0)
        assert np.array_equal(g2.get_x(), g.get_x())
    # problems of different kernel shapes cannot share a launch: branch mode
    mixed = binding.Batch([setup(orc, w, binding.FP32)[0] for w in small_members()])
    assert not mixed.set_mode(binding.BATCH_FUSED)
    # a few small volumes: the automatic mode fuses
    assert b.set_mode(binding.BATCH_AUTO)


def test_batch_fp64_matches_oracle(orc):
    ws = small_members()[:3]
    made = [setup(orc, w, binding.FP64) for w in ws]
    b = binding.Batch([m[0] for m in made])
    b.run(9)
    for (g, o, y), w in zip(made, ws):
        nc, order, _ = g.get_schedule()
        x = y.copy()
        d = np.zeros(w.shape)
        o.run(x, d, w.nslices, order, 9, history=False)
        assert rel(g.get_x(), x) <= 1e-11


def test_batch_stops_converged_problems(orc):
    ws = small_members()[:3]
    made = [setup(orc, w, binding.FP64) for w in ws]
    b = binding.Batch([m[0] for m in made])
    res = b.run(400, grad_rtol=1e-3, check_every=4)
    for (g, o, y), w, r in zip(made, ws, res):
        assert r["converged"] == 1
        assert r["grad_norm"] <= 1e-3 * r["grad_norm_ref"]
        assert r["sweeps"] % 4 == 0 and r["sweeps"] < 400
        # same state as a single run of that many sweeps
        g2 = setup(orc, w, binding.FP64)[0]
        g2.run(r["sweeps"], check_every=0)
        assert np.array_equal(g2.get_x(), g.get_x())


def test_batched_uneven_volumes_full_size(orc):
    """The 16-problem batch (128..256 x 128..256 x 32..96, PSF 7x7x7, 4..16
    blocks), tuned and run for 50 sweeps: equal to single runs with the same
    tile heights, and the three smallest problems against the oracle."""
    ws = [inputs.batch_member(p) for p in range(16)]
    made = [setup(orc, w, binding.FP32) for w in ws]
    probs = [m[0] for m in made]
    b = binding.Batch(probs)
    assert b.set_mode(binding.BATCH_FUSED)  # this batch can share launches
    b.tune()
    res = b.run(50)
    assert all(r["sweeps"] == 50 for r in res)
    nvox = sum(int(np.prod(w.shape)) for w in ws)
    print("fused batch: %d volumes, %d voxels, 50 sweeps in %.4f s: %.3e voxel-iterations/s"
          % (len(ws), nvox, res[0]["seconds"], nvox * 50 / res[0]["seconds"]))
    # 146 MB of volumes: the automatic mode takes graph branches
    assert not b.set_mode(binding.BATCH_AUTO)
    # single runs (tile heights as tuned) give the same iterates
    for i in (0, 7, 15):
        g = probs[i]
        xb = g.get_x()
        g.set_x0(None)
        g.run(50, check_every=0)
        assert np.array_equal(g.get_x(), xb), i
    # the three smallest problems against the FP64 oracle (3 sweeps)
    for i in np.argsort([np.prod(w.shape) for w in ws])[:3]:
        g, o, y = made[i]
        g.set_x0(None)
        g.run(3, check_every=0)
        nc, order, _ = g.get_schedule()
        x = y.copy()
        d = np.zeros(ws[i].shape)
        o.run(x, d, ws[i].nslices, order, 3, history=False)
        assert rel(g.get_x(), x) <= 2e-5, i
