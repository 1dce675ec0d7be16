"""Full-size parity: the 256x256x64 FP32 workload (the benchmark's volume, PSF
and partition) solved on the GPU, against the minimiser x* that the FP64
oracle alone computed to ||grad f|| <= 1e-9 ||grad f(y)|| (13500 sweeps;
tests/golden/plain_fp32_256x256x64.json, written by
tests/golden/make_golden.py; x* is stored at 4096 seeded voxels).

Both sides use the same inputs: y and the PSF factors formed with the oracle
and rounded to FP32 once.

* FP64 on the GPU to the oracle's tolerance 1e-9 reaches x* within 1e-6
  (relative, sampled) and f* within 1e-12, and stops in the same 250-sweep
  window as the oracle's recorded history.
* FP32 to the stopping tolerance 1e-6 (coloured and asynchronous-round
  schedules): f within 1e-7 of f*.  x is then as far from x* as the gradient
  tolerance allows, not closer: f is very flat along some directions (edges,
  where the TV weight is small), and the FP64 run stopped at the same 1e-6 is
  8.1e-4 from x*; reaching 1e-5 takes a gradient tolerance near 1e-8, below
  the FP32 floor (||grad f(fl32(x*))|| = 3.9e-7 ||grad f(y)||).  The FP32 bound
  on x at the stop is 1e-3 (measured 5.5e-4 coloured, 7.3e-4 in rounds; the
  FP64 iterate at the same gradient ratio is 5.5e-4 from x*).
* FP64 trajectory: x* is the oracle's iterate after its last recorded sweep
  count; the GPU's FP64 iterate after the same number of sweeps equals it
  within 1e-12 (rounding order only; measured about 1e-15).
* The 1e-5 target on x with single precision first: FP32 to 1e-6, its
  iterate and previous steps carried into an FP64 problem on the same inputs
  (residual rebuilt from x), FP64 on to 1e-8: x within 1e-5 of x* (measured
  9.8e-6) and f within 1e-12; the FP64 stage needs fewer sweeps than the
  FP32 one took.
* FP32 floor, run far past the 1e-6 stop (13500 sweeps, where FP64 reaches
  1e-9): the gradient ratio stays near the rounding floor (measured 4.5e-7,
  bound 2x the stored floor) and x stays 2.4e-4 from x* (bound 4e-4; 2.1e-4
  after 20000 sweeps): single precision storage cannot reach the 1e-5
  target on x, whatever the sweep count; f is within 1e-9 of f*.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2002_02328_amd import binding, inputs

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "plain_fp32_256x256x64.json")


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def golden():
    if not os.path.exists(GOLD):
        pytest.skip("stored minimiser not generated")
    with open(GOLD) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def data(golden):
    w = inputs.mid_fp32()
    assert w.name == golden["workload"]
    gxy = f32(oracle.gauss_table(w.sigma_xy, w.kxy))
    gz = f32(oracle.gauss_table(w.sigma_z, w.kz))
    y = f32(oracle.Problem(np.zeros(w.shape), gxy, gxy, gz).H(w.xbar) + w.noise)
    return w, gxy, gz, y


def solve(data, prec, schedule, tol, sweeps=40000):
    """Run to the tolerance (tol > 0) or exactly `sweeps` sweeps (tol = 0,
    then f and ||grad f|| are evaluated at the end)."""
    w, gxy, gz, y = data
    nz, ny, nx = w.shape
    g = binding.Problem(nx, ny, nz, prec)
    g.set_psf_separable(gxy, gxy, gz)
    g.set_params(w.lam, w.delta, w.eta, w.kappa)
    g.set_data(y.astype(g.dtype))
    g.set_blocks(w.nslices, schedule)
    g.set_x0(None)
    if tol > 0:
        res = g.run(sweeps, grad_rtol=tol, check_every=1)
    else:
        res = g.run(sweeps, check_every=sweeps)
    x = g.get_x().astype(np.float64).ravel()
    g.close()
    return res, x


def errors(golden, res, x):
    idx = np.asarray(golden["sample_index"])
    xs = np.asarray(golden["sample_x"])
    ex = np.linalg.norm(x[idx] - xs) / np.linalg.norm(xs)
    ef = abs(res["f"] - golden["f_star"]) / abs(golden["f_star"])
    return ex, ef


def test_fp64_reaches_the_oracle_minimiser(golden, data):
    res, x = solve(data, binding.FP64, binding.SCHED_COLORED, 1e-9)
    assert res["converged"]
    assert abs(res["grad_norm_ref"] - golden["grad_ref"]) <= 1e-9 * golden["grad_ref"]
    ex, ef = errors(golden, res, x)
    print("FP64 to 1e-9: %d sweeps, |x - x*| / |x*| = %.3e, |f - f*| / f* = %.3e" % (res["sweeps"], ex, ef))
    assert ex <= 1e-6 and ef <= 1e-12
    # the oracle's history brackets the sweep where 1e-9 is crossed
    hist = golden["history"]
    before = max(s for s, r in hist if r > 1e-9)
    after = min(s for s, r in hist if r <= 1e-9)
    assert before < res["sweeps"] <= after


@pytest.mark.parametrize("schedule", [binding.SCHED_COLORED, binding.SCHED_ROUND])
def test_fp32_stop_tolerance_against_oracle_minimiser(golden, data, schedule):
    res, x = solve(data, binding.FP32, schedule, 1e-6)
    assert res["converged"]
    assert abs(res["grad_norm_ref"] - golden["grad_ref"]) <= 1e-5 * golden["grad_ref"]
    ex, ef = errors(golden, res, x)
    print("FP32 schedule %d to 1e-6: %d sweeps, |x - x*| / |x*| = %.3e, |f - f*| / f* = %.3e"
          % (schedule, res["sweeps"], ex, ef))
    assert ef <= 1e-7
    assert ex <= 1e-3


def test_fp64_trajectory_equals_the_oracle_run(golden, data):
    res, x = solve(data, binding.FP64, binding.SCHED_COLORED, 0.0, sweeps=golden["sweeps"])
    ex, ef = errors(golden, res, x)
    print("FP64, %d sweeps: |x - x_oracle| / |x_oracle| = %.3e" % (golden["sweeps"], ex))
    assert ex <= 1e-12 and ef <= 1e-13


def test_fp32_floor_far_past_the_stop_tolerance(golden, data):
    res, x = solve(data, binding.FP32, binding.SCHED_COLORED, 0.0, sweeps=13500)
    ex, ef = errors(golden, res, x)
    gr = res["grad_norm"] / golden["grad_ref"]
    print("FP32, 13500 sweeps: ||grad f|| / ||grad f(y)|| = %.3e, |x - x*| / |x*| = %.3e, "
          "|f - f*| / f* = %.3e" % (gr, ex, ef))
    assert gr <= 2 * golden["fp32_floor_grad_ratio"]
    assert ex <= 4e-4
    assert ef <= 1e-9


def test_fp32_then_fp64_reaches_the_x_target(golden, data):
    w, gxy, gz, y = data
    nz, ny, nx = w.shape
    g = binding.Problem(nx, ny, nz, binding.FP32)
    g.set_psf_separable(gxy, gxy, gz)
    g.set_params(w.lam, w.delta, w.eta, w.kappa)
    g.set_data(y.astype(np.float32))
    g.set_blocks(w.nslices)
    g.set_x0(None)
    r1 = g.run(40000, grad_rtol=1e-6, check_every=binding.CHECK_ADAPTIVE)
    assert r1["converged"]
    x, d, q, sw = g.get_state()
    g.close()
    h = binding.Problem(nx, ny, nz, binding.FP64)
    h.set_psf_separable(gxy, gxy, gz)
    h.set_params(w.lam, w.delta, w.eta, w.kappa)
    h.set_data(y)
    h.set_blocks(w.nslices)
    h.get_schedule()
    h.set_state(x.astype(np.float64), d.astype(np.float64), None, sw)
    r2 = h.run(40000, grad_rtol=1e-8, check_every=binding.CHECK_ADAPTIVE)
    assert r2["converged"]
    assert abs(r2["grad_norm_ref"] - golden["grad_ref"]) <= 1e-9 * golden["grad_ref"]
    ex, ef = errors(golden, r2, h.get_x().astype(np.float64).ravel())
    print("FP32 %d sweeps to 1e-6, then FP64 %d sweeps to 1e-8: |x - x*| / |x*| = %.3e, |f - f*| / f* = %.3e"
          % (r1["sweeps"], r2["sweeps"], ex, ef))
    h.close()
    assert ex <= 1e-5 and ef <= 1e-12
    assert r2["sweeps"] < 2 * r1["sweeps"]
