"""Full-size parity: the 256x256x64 FP32 workload (the benchmark's volume, PSF
and partition) solved on the GPU, against the minimiser x* that the FP64
oracle alone computed to ||grad f|| <= 1e-9 ||grad f(y)||
(tests/golden/plain_fp32_256x256x64.json, written by tests/golden/make_golden.py;
x* is stored at 4096 seeded voxels).

Both sides use the same inputs: y and the PSF factors formed with the oracle
and rounded to FP32 once.  The GPU runs to its stopping tolerance 1e-6 under
the coloured and the asynchronous-round schedules.  Bounds (the accuracy
targets of the workload): x within 1e-5 of x* in relative norm on the sampled
voxels and f within 1e-7 of f*, relative.
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


@pytest.mark.parametrize("schedule", [binding.SCHED_COLORED, binding.SCHED_ROUND])
def test_fp32_solution_matches_oracle_minimiser(golden, data, schedule):
    w, gxy, gz, y = data
    nz, ny, nx = w.shape
    g = binding.Problem(nx, ny, nz, binding.FP32)
    g.set_psf_separable(gxy, gxy, gz)
    g.set_params(w.lam, w.delta, w.eta, w.kappa)
    g.set_data(y.astype(np.float32))
    g.set_blocks(w.nslices, schedule)
    g.set_x0(None)
    res = g.run(20000, grad_rtol=1e-6, check_every=1)
    assert res["converged"]
    assert abs(res["grad_norm_ref"] - golden["grad_ref"]) <= 1e-5 * golden["grad_ref"]
    x = g.get_x().astype(np.float64).ravel()
    idx = np.asarray(golden["sample_index"])
    xs = np.asarray(golden["sample_x"])
    ex = np.linalg.norm(x[idx] - xs) / np.linalg.norm(xs)
    ef = abs(res["f"] - golden["f_star"]) / abs(golden["f_star"])
    print("schedule %d: %d sweeps, |x - x*| / |x*| = %.3e (sampled), |f - f*| / f* = %.3e"
          % (schedule, res["sweeps"], ex, ef))
    assert ex <= 1e-5
    assert ef <= 1e-7
    g.close()
