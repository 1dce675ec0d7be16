"""The committed warm-start weights (paper_2002_02328_amd/weights) against the
problems they are meant for.

* On a held-out training-distribution volume (pair 1999 of the trainer's 2000,
  one of the 100 it validates on and never fits), x0 = y + net(y) is much
  closer to the BD3MG solution than y is.
* On a fresh 256x256x64 volume, BD3MG started from x0 reaches the gradient
  tolerances 1e-4 and 1e-6 (relative to ||grad f(y)||, the same normaliser for
  both starts) in fewer sweeps than from y, and to the same minimum.
"""
import os

import numpy as np
import pytest

from paper_2002_02328_amd import binding, inputs
from paper_2002_02328_amd.train_warmstart import WEIGHTS, make_problem, time_to_tol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def net():
    assert os.path.exists(WEIGHTS), "trained weights missing"
    n = binding.Net()
    n.load(open(WEIGHTS, "rb").read())
    yield n
    n.close()


def test_network_moves_y_towards_the_solution(net):
    w = inputs.warmstart_train_member(1999)
    p, y = make_problem(w)
    res = p.run(3000, grad_rtol=1e-4, check_every=8)
    assert res["converged"]
    xs = p.get_x().astype(np.float64)
    x0 = net.forward(y).astype(np.float64)
    e_net = np.mean((x0 - xs) ** 2)
    e_y = np.mean((y.astype(np.float64) - xs) ** 2)
    print("held-out pair: mse(x0, x*) = %.3e, mse(y, x*) = %.3e" % (e_net, e_y))
    assert e_net < 0.2 * e_y
    p.close()


@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_warm_start_needs_fewer_sweeps(net, tol):
    w = inputs.warmstart_eval_member(0)
    plain = time_to_tol(w, None, tol)
    warm = time_to_tol(w, net, tol, tiles=plain["tile_rows"])
    print("tol %.0e: plain %d sweeps %.3f s, warm %d sweeps %.3f s (inference %.4f s)"
          % (tol, plain["sweeps"], plain["seconds"], warm["sweeps"], warm["seconds"], warm["infer_seconds"]))
    assert plain["converged"] and warm["converged"]
    assert warm["sweeps"] < plain["sweeps"]
    # both reach the same minimum (f is strictly convex)
    assert abs(warm["f"] - plain["f"]) <= 10 * tol * abs(plain["f"])
