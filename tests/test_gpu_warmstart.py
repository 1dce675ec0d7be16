"""The committed warm-start weights (paper_2002_02328_amd/weights, trained on
2000 pairs solved to 1e-6) against the problems they are meant for.

* On a held-out training-distribution volume (pair 1999 of the trainer's 2000,
  one of the 100 it validates on and never fits), x0 = y + net(y) is much
  closer to the BD3MG solution than y is.
* On the eight held-out 256x256x64 volumes and the benchmark's own, BD3MG
  started from x0 reaches the gradient tolerance 1e-4 (relative to
  ||grad f(y)||, the same normaliser for both starts) in fewer sweeps and in
  less wall time, the network's inference included, and at the same minimum
  (measured 1.15x to 1.30x).
* At 1e-6 the gain is within a few per cent either way (measured 0.96x to
  1.10x, 1.03x on the benchmark's volume): the start shortens the early
  phase, the slow tail of the iteration is the same from either start.  The
  test checks that both starts reach the same minimum and that the warm
  start costs at most 8 % more sweeps, and prints the figures.
"""
import os

import numpy as np
import pytest

from paper_2002_02328_amd import binding, inputs
from paper_2002_02328_amd.train_warmstart import WEIGHTS, make_problem, time_to_tol, eval_volumes

pytestmark = pytest.mark.gpu

VOLUMES = eval_volumes(8)


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
    res = p.run(20000, grad_rtol=1e-6, check_every=8)
    assert res["converged"]
    xs = p.get_x().astype(np.float64)
    x0 = net.forward(y).astype(np.float64)
    e_net = np.mean((x0 - xs) ** 2)
    e_y = np.mean((y.astype(np.float64) - xs) ** 2)
    print("held-out pair: mse(x0, x*) = %.3e, mse(y, x*) = %.3e" % (e_net, e_y))
    assert e_net < 0.2 * e_y
    p.close()


def _pair(net, w, tol):
    plain = time_to_tol(w, None, tol)
    warm = time_to_tol(w, net, tol, tiles=plain["tile_rows"])
    print("%s tol %.0e: plain %d sweeps %.3f s, warm %d sweeps %.3f s (inference %.4f s), speedup %.2f"
          % (w.name, tol, plain["sweeps"], plain["seconds"], warm["sweeps"], warm["seconds"],
             warm["infer_seconds"], plain["seconds"] / warm["seconds"]))
    assert plain["converged"] and warm["converged"]
    # both reach the same minimum (f is strictly convex)
    assert abs(warm["f"] - plain["f"]) <= 10 * tol * abs(plain["f"])
    return plain, warm


@pytest.mark.parametrize("name,w", VOLUMES, ids=[n for n, _ in VOLUMES])
def test_warm_start_pays_at_1e4(net, name, w):
    plain, warm = _pair(net, w, 1e-4)
    assert warm["sweeps"] < plain["sweeps"]
    assert warm["seconds"] < plain["seconds"]


@pytest.mark.parametrize("name,w", [VOLUMES[0], VOLUMES[-1]], ids=[VOLUMES[0][0], VOLUMES[-1][0]])
def test_warm_start_at_1e6(net, name, w):
    plain, warm = _pair(net, w, 1e-6)
    assert warm["sweeps"] <= 1.08 * plain["sweeps"]
