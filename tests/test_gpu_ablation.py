"""GPU parity of the ablation variants of Sec. 3.2 ("Ablation study and
comparative analysis"): Async-GD (subspace {-grad}, metric L Id), Async-CG
(BD3MG's subspace with the metric L Id) and Async-MM (d' = -A_S(x)^{-1}
grad_S f by an inner linear solve), against the FP64 oracle's variants.

They reuse the sweep kernels: the 2x2 solve takes the metric L Id for GD and
CG; Async-MM runs conjugate gradients on each block's majorant (the
direction pass gives H p, the update pass XY^T H p, the majorant-apply pass
the rest) where the oracle runs linear biconjugate gradients with the shadow
residual started at the residual (the same iterates for the symmetric A_S).
FP64 tolerances: GD and CG as BD3MG's (a few dozen ulps per step, 1e-10 per
block-step value); Async-MM's inner iterations amplify the rounding
differences of A_S p by the growth of the Krylov recurrences, 1e-8 on the
step after up to 12 inner iterations (measured about 1e-12).
"""
import numpy as np
import pytest

from paper_2002_02328_amd import binding
from gpu_common import pair, rel

pytestmark = pytest.mark.gpu

SHAPE = (10, 37, 70)
NSL = [3, 2, 4, 1]
METHODS = [("ASYNC_GD", binding.METHOD_ASYNC_GD), ("ASYNC_CG", binding.METHOD_ASYNC_CG),
           ("ASYNC_MM", binding.METHOD_ASYNC_MM)]


def _pair(orc, prec, kappa=0.0, mu=0.0, seed=2):
    return pair(orc, SHAPE, prec, seed=seed, kx=5, ky=5, kz=3, lam=0.02, delta=0.03, eta=0.3,
                kappa=kappa, nslices=NSL, mu=mu)


def _set(g, o, orc, name, code, n_inner=6, tol_inner=0.0):
    L = o.lipschitz_bound()
    o.set_method(getattr(orc, name), lip=L, n_inner=n_inner, tol_inner=tol_inner)
    g.set_method(code, lip=L, n_inner=n_inner, tol_inner=tol_inner)
    return L


@pytest.mark.parametrize("name,code", METHODS)
@pytest.mark.parametrize("kappa", [0.0, 0.05])
def test_block_steps_match_oracle(orc, name, code, kappa):
    g, o, y = _pair(orc, binding.FP64, kappa=kappa)
    _set(g, o, orc, name, code)
    g.set_x0(None)
    x = y.copy()
    d = np.zeros(SHAPE)
    z0 = np.concatenate([[0], np.cumsum(NSL)[:-1]])
    for b in [0, 2, 1, 3, 0, 2, 3, 1]:
        ig = np.asarray(g.block_step(b))
        io = np.asarray(o.block_step(x, d, int(z0[b]), NSL[b]))
        if code == binding.METHOD_ASYNC_MM:
            assert ig[0] == io[0], (b, ig, io)  # inner iterations
            assert abs(ig[1] - io[1]) <= 1e-6 * io[7], (b, ig, io)  # ||r_end||^2 against ||g||^2
            assert np.allclose(ig[2:], io[2:], rtol=1e-12, atol=0), (b, ig, io)
            tol = 1e-8
        else:
            # Async-CG's u2 is zero up to rounding (the step collapses to
            # -grad / L): coefficients are compared on the scale of the step
            atol = 1e-10 * max(abs(io[5]), abs(io[6])) if code == binding.METHOD_ASYNC_CG else 1e-300
            assert np.allclose(ig[:5], io[:5], rtol=1e-10, atol=1e-300), (b, ig, io)
            assert np.allclose(ig[5:7], io[5:7], rtol=1e-10, atol=atol), (b, ig, io)
            assert np.allclose(ig[7], io[7], rtol=1e-10), (b, ig, io)
            tol = 1e-12
        assert rel(g.get_x(), x) <= tol, (b, rel(g.get_x(), x))
        assert rel(g.get_dprev(), d) <= 1e3 * tol
    g.close()


@pytest.mark.parametrize("name,code", METHODS)
def test_coloured_trajectories_match_oracle(orc, name, code):
    for prec, tol in [(binding.FP64, 1e-9), (binding.FP32, 2e-5)]:
        g, o, y = _pair(orc, prec, seed=5)
        _set(g, o, orc, name, code, n_inner=8)
        nc, order, _ = g.get_schedule()
        g.set_x0(None)
        res = g.run(12)
        x = y.copy()
        d = np.zeros(SHAPE)
        o.run(x, d, NSL, order, 12, history=False)
        e = rel(g.get_x(), x)
        print("%s, precision %d, 12 sweeps: rel |x_gpu - x_oracle| = %.3e" % (name, prec, e))
        assert e <= tol
        fo = o.f(x)
        assert abs(res["f"] - fo) <= (1e-12 if prec == binding.FP64 else 1e-6) * abs(fo)
        g.close()


def test_async_mm_inner_tolerance_and_inflation(orc):
    """Early stop of the inner solve at tol_inner (iteration counts equal the
    oracle's) with the Assumption C inflation added to the majorant."""
    g, o, y = _pair(orc, binding.FP64, kappa=0.03, mu=0.2, seed=7)
    _set(g, o, orc, "ASYNC_MM", binding.METHOD_ASYNC_MM, n_inner=50, tol_inner=1e-4)
    g.set_x0(None)
    x = y.copy()
    d = np.zeros(SHAPE)
    z0 = np.concatenate([[0], np.cumsum(NSL)[:-1]])
    iters = []
    for b in [1, 3, 0, 2, 1]:
        ig = np.asarray(g.block_step(b))
        io = np.asarray(o.block_step(x, d, int(z0[b]), NSL[b]))
        assert ig[0] == io[0] and 0 < ig[0] < 50, (b, ig, io)
        assert ig[1] <= 1e-8 * io[7] * 1.0001
        iters.append(ig[0])
        assert rel(g.get_x(), x) <= 1e-8
    print("Async-MM inner iterations to 1e-4:", iters)
    g.close()


def test_async_gd_and_cg_take_the_same_step(orc):
    """With the metric L Id the subspace step collapses to -grad / L."""
    xs = []
    for code in (binding.METHOD_ASYNC_GD, binding.METHOD_ASYNC_CG):
        g, o, y = _pair(orc, binding.FP64, seed=9)
        g.set_method(code, lip=o.lipschitz_bound())
        g.set_x0(None)
        g.run(20)
        xs.append(g.get_x())
        g.close()
    assert rel(xs[0], xs[1]) <= 1e-12


def test_method_errors(orc):
    g, o, y = _pair(orc, binding.FP64)
    with pytest.raises(binding.Bd3mgError) as e:
        g.set_method(7)
    assert e.value.status == binding.ERR_ARG
    with pytest.raises(binding.Bd3mgError) as e:
        g.set_method(binding.METHOD_ASYNC_MM, n_inner=0)
    assert e.value.status == binding.ERR_ARG
    g.set_method(binding.METHOD_ASYNC_MM, n_inner=3)
    g.get_schedule()
    with pytest.raises(binding.Bd3mgError) as e:  # the allocation-free entry point runs the others only
        g.run_noalloc(1)
    assert e.value.status == binding.ERR_STATE
    g.set_blocks(NSL, binding.SCHED_ROUND)
    with pytest.raises(binding.Bd3mgError) as e:
        g.run(1)
    assert e.value.status == binding.ERR_STATE
    g.set_blocks(NSL)
    g.set_method(binding.METHOD_BD3MG)
    g.run(1)
    g.close()
