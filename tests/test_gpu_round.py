"""GPU parity of the asynchronous-round schedule (BD3MG_SCHED_ROUND: every
block steps from the same snapshot, Sec. 2.4) and of the curvature inflation
(Assumption C) against the FP64 oracle's run_round / run.

Tolerances as in test_gpu_solver: FP64 trajectories within 1e-9 relative
(differences in summation order only), FP32 within 2e-4 of the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2002_02328_amd import binding, inputs
from gpu_common import rel, rounded

pytestmark = pytest.mark.gpu


def setup(shape, seed, prec, kxy, kz, nslices, schedule, mu=0.0, sigma_z=(2.0, 2.0), kappa=0.0):
    nz, ny, nx = shape
    w = inputs.tiny(shape, seed, kxy=kxy, kz=kz, nblocks=len(nslices), sigma_z=sigma_z,
                    lam=0.01, delta=0.05, eta=0.01, kappa=kappa)
    gxy = rounded(oracle.gauss_table(w.sigma_xy, w.kxy), prec)
    gz = rounded(oracle.gauss_table(w.sigma_z, w.kz), prec)
    y = rounded(oracle.Problem(np.zeros(shape), gxy, gxy, gz).H(w.xbar) + w.noise, prec)
    o = oracle.Problem(y, gxy, gxy, gz, lam=w.lam, delta=w.delta, eta=w.eta, kappa=w.kappa, mu=mu)
    g = binding.Problem(nx, ny, nz, prec)
    g.set_psf_separable(gxy, gxy, gz)
    g.set_params(w.lam, w.delta, w.eta, w.kappa)
    g.set_inflation(mu)
    g.set_data(y)
    g.set_blocks(np.asarray(nslices, np.int32), schedule)
    g.set_x0(None)
    return g, o, y


@pytest.mark.parametrize("shape,nslices,kxy,kz,mu,kappa", [
    ((8, 16, 16), [2, 2, 2, 2], 3, 5, 0.0, 0.0),
    ((9, 21, 70), [1, 3, 2, 3], 5, 7, 0.5, 0.0),
    ((12, 33, 65), [4, 1, 1, 6], 7, 3, 0.2, 0.0),
    ((10, 19, 37), [3, 2, 1, 4], 9, 9, 0.3, 0.05),
    ((1, 30, 50), [1], 5, 1, 0.0, 0.0),
    ((5, 7, 9), [1, 1, 1, 1, 1], 3, 3, 0.1, 0.02),
])
def test_round_trajectory_fp64(orc, shape, nslices, kxy, kz, mu, kappa):
    g, o, y = setup(shape, 5, binding.FP64, kxy, kz, nslices, binding.SCHED_ROUND, mu, kappa=kappa)
    nc, order, color = g.get_schedule()
    assert nc == 1 and list(color) == [0] * len(nslices)
    x, d = y.copy(), np.zeros(shape)
    done = 0
    for cp in (1, 5, 30):
        res = g.run(cp - done)
        o.run_round(x, d, nslices, cp - done, history=False)
        done = cp
        assert rel(g.get_x(), x) <= 1e-9, cp
        # near convergence the last step is tiny: bound its error by the
        # iterate's scale as well
        dd = np.linalg.norm(g.get_dprev() - d)
        assert dd <= 1e-9 * np.linalg.norm(d) + 1e-13 * np.linalg.norm(x), cp
        assert abs(res["f"] - o.f(x)) <= 1e-12 * abs(o.f(x))


def test_colored_schedule_with_inflation_fp64(orc):
    nslices = [2, 3, 1, 4, 2]
    g, o, y = setup((12, 20, 40), 6, binding.FP64, 5, 5, nslices, binding.SCHED_COLORED, mu=0.7)
    nc, order, color = g.get_schedule()
    x, d = y.copy(), np.zeros(y.shape)
    g.run(12)
    o.run(x, d, nslices, order, 12, history=False)
    assert rel(g.get_x(), x) <= 1e-9


def test_round_fp32_tracks_fp64_oracle(orc):
    nslices = [2, 2, 3, 1, 2]
    g, o, y = setup((10, 40, 72), 7, binding.FP32, 5, 7, nslices, binding.SCHED_ROUND, mu=0.5)
    x, d = y.copy(), np.zeros(y.shape)
    g.run(25)
    o.run_round(x, d, nslices, 25, history=False)
    assert rel(g.get_x(), x) <= 2e-4


def test_round_stop_rule_matches_oracle(orc):
    nslices = [2, 2, 2, 2]
    g, o, y = setup((8, 16, 16), 8, binding.FP64, 3, 5, nslices, binding.SCHED_ROUND)
    res = g.run(500, grad_rtol=1e-4, check_every=1)
    x, d = y.copy(), np.zeros(y.shape)
    s, fh, gh = o.run_round(x, d, nslices, 500, grad_rtol=1e-4)
    assert res["converged"] == 1 and res["sweeps"] == s


@pytest.mark.parametrize("prec,tol", [(binding.FP64, 1e-14), (binding.FP32, 1e-6)])
def test_lipschitz_bound_matches_oracle(orc, prec, tol):
    g, o, y = setup((9, 16, 24), 9, prec, 5, 7, [3, 3, 3], binding.SCHED_ROUND)
    assert abs(g.lipschitz_bound() - o.lipschitz_bound()) <= tol * o.lipschitz_bound()


def test_undelayed_round_diverges_and_inflation_descends(orc):
    """Thin blocks under a wide z blur: without inflation the round overshoots
    (f grows); with mu = L (2 sqrt(tau) + 1) from the library's own bound,
    f decreases monotonically."""
    nslices = [2] * 8
    g, o, y = setup((16, 24, 24), 5, binding.FP64, 3, 7, nslices, binding.SCHED_ROUND)
    f0 = o.f(y)
    res = g.run(40)
    assert res["f"] > 10 * f0
    L = g.lipschitz_bound()
    g.set_inflation(L * (2 * np.sqrt(len(nslices) - 1) + 1))
    g.set_x0(None)
    prev = f0
    for _ in range(8):
        f = g.run(5)["f"]
        assert f <= prev * (1 + 1e-13)
        prev = f
    assert prev < f0


def test_round_batch_equals_single_runs(orc):
    cases = [((8, 16, 16), [2, 2, 2, 2], 3, 5), ((9, 21, 70), [1, 3, 2, 3], 5, 7)]
    single = []
    for i, (shape, ns, kxy, kz) in enumerate(cases):
        g, o, y = setup(shape, 20 + i, binding.FP32, kxy, kz, ns, binding.SCHED_ROUND, mu=0.3)
        g.run(7, check_every=0)
        single.append(g.get_x())
    probs = [setup(shape, 20 + i, binding.FP32, kxy, kz, ns, binding.SCHED_ROUND, mu=0.3)[0]
             for i, (shape, ns, kxy, kz) in enumerate(cases)]
    b = binding.Batch(probs)
    b.run(7)
    for g, xs in zip(probs, single):
        assert np.array_equal(g.get_x(), xs)


@pytest.mark.parametrize("schedule", [binding.SCHED_COLORED, binding.SCHED_ROUND])
@pytest.mark.parametrize("prec", [binding.FP64, binding.FP32])
@pytest.mark.parametrize("kz", [7, 1])
def test_direction_slices_per_workgroup_bitwise(orc, schedule, prec, kz):
    """Two output slices per direction workgroup (their common source slices
    read once) give bitwise the result of one slice per workgroup; blocks with
    odd and even numbers of direction slices, kappa > 0 (the VZ sums), and the
    FP64 trajectory of the paired pass against the oracle."""
    nslices = [3, 1, 4, 2, 5]
    runs = []
    for per in (1, 2):
        g, o, y = setup((15, 20, 70), 11, prec, 5, kz, nslices, schedule, mu=0.2, kappa=0.03)
        g.set_option(binding.OPT_DIRS_SLICES, per)
        g.run(6)
        runs.append((g.get_x(), g.get_dprev()))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    if prec == binding.FP64:
        x, d = y.copy(), np.zeros(y.shape)
        if schedule == binding.SCHED_ROUND:
            o.run_round(x, d, nslices, 6, history=False)
        else:
            nc, order, color = g.get_schedule()
            o.run(x, d, nslices, order, 6, history=False)
        assert rel(runs[1][0], x) <= 1e-9


def test_guard_restores_and_raises_the_inflation(orc):
    """The divergent case above (thin blocks, wide z blur, mu = 0) with the
    guard every 4 sweeps: the guard restores the last accepted state at
    least once and raises mu within (0, L (2 sqrt(tau) + 1)]; f after every
    guarded call is at most f before it (up to the guard's FP64 slack); the
    run ends below f(y); discarded sweeps are counted in the call's sweeps
    but not in the state's sweep count."""
    nslices = [2] * 8
    g, o, y = setup((16, 24, 24), 5, binding.FP64, 3, 7, nslices, binding.SCHED_ROUND)
    f0 = o.f(y)
    g.set_option(binding.OPT_ROUND_GUARD, 4)
    prev, trips_total = f0, 0
    for _ in range(10):
        r = g.run(8)
        trips, mu = g.round_guard_info()
        trips_total += trips
        assert r["sweeps"] == 8
        assert r["f"] <= prev * (1 + 1e-13)
        prev = r["f"]
    L = g.lipschitz_bound()
    print("guard: %d restores, mu = %.4g (cap %.4g), f %.6g -> %.6g, state sweeps %d of 80"
          % (trips_total, mu, L * (2 * np.sqrt(7) + 1), f0, prev, g.get_state()[3]))
    assert trips_total >= 1
    assert 0 < mu <= L * (2 * np.sqrt(len(nslices) - 1) + 1) * (1 + 1e-12)
    assert prev < f0
    assert g.get_state()[3] < 80


def test_guard_leaves_a_converging_round_unchanged(orc):
    """Where the rounds descend, the guard accepts every check: the iterate
    is bitwise that of the unguarded run and mu is untouched."""
    out = []
    for m in (0, 4):
        g, o, y = setup((9, 21, 70), 21, binding.FP32, 5, 7, [1, 3, 2, 3], binding.SCHED_ROUND, mu=0.3)
        g.set_option(binding.OPT_ROUND_GUARD, m)
        r = g.run(24, check_every=0)
        trips, mu = g.round_guard_info()
        assert trips == 0 and mu == 0.3 and r["sweeps"] == 24 and g.get_state()[3] == 24
        out.append((g.get_x(), g.get_dprev()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
