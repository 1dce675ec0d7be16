"""Pins of the oracle's asynchronous rounds (every block steps from the same
snapshot, Sec. 2.4) and of the curvature inflation of Assumption C, against
facts that do not come from the oracle:

* without coupling between blocks (no z blur, kappa = 0) or with one block, a
  round is exactly the sequential sweep;
* the round reaches the same minimiser as the sequential schedule (f is
  strictly convex);
* an inflation mu much larger than the curvature turns the step into
  steepest descent with step 1/mu;
* with thin blocks under a wide z blur the undelayed-majorant round
  overshoots and diverges, and the inflation that Assumption C asks for,
  mu = L (2 sqrt(tau) + 1) with tau = nblocks - 1, restores monotone descent;
* the Lipschitz bound of Assumption A bounds measured gradient differences.
"""
import numpy as np
import pytest

import oracle
from paper_2002_02328_amd import inputs


def problem(shape, seed, kxy, kz, nblocks, sigma_z=(2.0, 2.0), mu=0.0, lam=0.01, kappa=0.0):
    w = inputs.tiny(shape, seed, kxy=kxy, kz=kz, nblocks=nblocks, sigma_z=sigma_z, lam=lam,
                    delta=0.05, eta=0.01, kappa=kappa)
    gxy = oracle.gauss_table(w.sigma_xy, w.kxy)
    gz = oracle.gauss_table(w.sigma_z, w.kz)
    y = oracle.Problem(np.zeros(w.shape), gxy, gxy, gz).H(w.xbar) + w.noise
    o = oracle.Problem(y, gxy, gxy, gz, lam=w.lam, delta=w.delta, eta=w.eta, kappa=w.kappa, mu=mu)
    return o, y


def test_round_equals_sequential_without_coupling(orc):
    o, y = problem((8, 12, 16), 1, kxy=5, kz=1, nblocks=4)
    ns = np.array([1, 3, 2, 2], np.int32)
    xr, dr = y.copy(), np.zeros(y.shape)
    xs, ds = y.copy(), np.zeros(y.shape)
    o.run_round(xr, dr, ns, 5, history=False)
    o.run(xs, ds, ns, np.arange(4), 5, history=False)
    assert np.array_equal(xr, xs) and np.array_equal(dr, ds)


def test_single_block_round_equals_sequential(orc):
    o, y = problem((6, 10, 12), 2, kxy=3, kz=5, nblocks=1, mu=0.3)
    ns = np.array([6], np.int32)
    xr, dr = y.copy(), np.zeros(y.shape)
    xs, ds = y.copy(), np.zeros(y.shape)
    o.run_round(xr, dr, ns, 4, history=False)
    o.run(xs, ds, ns, [0], 4, history=False)
    assert np.array_equal(xr, xs)


def test_round_reaches_the_sequential_minimiser(orc):
    o, y = problem((8, 16, 16), 5, kxy=3, kz=5, nblocks=4)
    ns = np.full(4, 2, np.int32)
    xr, dr = y.copy(), np.zeros(y.shape)
    sr, _, gr = o.run_round(xr, dr, ns, 1000, grad_rtol=1e-9)
    xs, ds = y.copy(), np.zeros(y.shape)
    nc, order, _ = oracle.color_schedule(ns, 4)
    ss, _, gs = o.run(xs, ds, ns, order, 2000, grad_rtol=1e-9)
    assert gr[-1] <= 1e-9 * o.grad_norm(y) and gs[-1] <= 1e-9 * o.grad_norm(y)
    assert np.linalg.norm(xr - xs) <= 1e-6 * np.linalg.norm(xs)


def test_large_inflation_is_scaled_steepest_descent(orc):
    mu = 1e8
    o, y = problem((6, 12, 12), 3, kxy=3, kz=3, nblocks=3, mu=mu)
    ns = np.array([2, 2, 2], np.int32)
    x, d = y.copy(), np.zeros(y.shape)
    o.run_round(x, d, ns, 1, history=False)
    step = -o.grad(y) / mu
    assert np.linalg.norm((x - y) - step) <= 1e-6 * np.linalg.norm(step)


def test_undelayed_round_diverges_and_assumption_c_inflation_descends(orc):
    o, y = problem((16, 24, 24), 5, kxy=3, kz=7, nblocks=8)
    ns = np.full(8, 2, np.int32)
    x, d = y.copy(), np.zeros(y.shape)
    _, fh, _ = o.run_round(x, d, ns, 40)
    assert fh[-1] > 10 * o.f(y)  # overshoot grows without bound
    L = o.lipschitz_bound()
    mu = L * (2 * np.sqrt(ns.size - 1) + 1)
    oc = oracle.Problem(o.y, o.gx, o.gy, o.gz, lam=o.lam, delta=o.delta, eta=o.eta, kappa=o.kappa, mu=mu)
    x, d = y.copy(), np.zeros(y.shape)
    _, fh, _ = oc.run_round(x, d, ns, 40)
    seq = np.concatenate([[oc.f(y)], fh])
    assert np.all(np.diff(seq) <= 1e-13 * abs(seq[0]))
    assert fh[-1] < seq[0]


@pytest.mark.parametrize("kappa", [0.0, 0.05])
def test_lipschitz_bound_holds(orc, kappa):
    o, y = problem((6, 14, 18), 7, kxy=5, kz=5, nblocks=3, sigma_z=(0.6, 1.5), kappa=kappa, lam=0.2)
    L = o.lipschitz_bound()
    rng = np.random.default_rng(1)
    worst = 0.0
    for _ in range(10):
        a = rng.uniform(-0.5, 1.5, y.shape)
        b = a + rng.standard_normal(y.shape) * 10.0 ** rng.uniform(-3, 0)
        worst = max(worst, np.linalg.norm(o.grad(a) - o.grad(b)) / np.linalg.norm(a - b))
    # a small in-slice checkerboard on a flat volume excites the TV term at
    # its largest curvature, 8 lambda / delta
    nz, ny, nx = y.shape
    cb = np.fromfunction(lambda k, j, i: (-1.0) ** (i + j), y.shape)
    a = np.full(y.shape, 0.5)
    r = np.linalg.norm(o.grad(a + 1e-4 * cb) - o.grad(a)) / np.linalg.norm(1e-4 * cb)
    assert r >= 0.5 * 8 * o.lam / o.delta
    worst = max(worst, r)
    assert worst <= L
    # data term alone: the bound is within a factor 2 of ||H^T H|| (power iteration)
    od = oracle.Problem(o.y, o.gx, o.gy, o.gz)
    v = rng.standard_normal(y.shape)
    for _ in range(60):
        v = od.HT(od.H(v))
        nrm = np.linalg.norm(v)
        v /= nrm
    assert nrm <= od.lipschitz_bound() <= 2 * nrm
