"""GPU parity of the warm-start network (bd3mg_net_*) against the FP64 oracle
of convnet_oracle.c run with bfloat16 storage emulation.

Tolerances.  Both sides round the same activations and weights to bfloat16;
they differ in the order and precision of the sums (float on the matrix
cores, FP64 in the oracle), so a sum that lands within about 2^-20 of a
bfloat16 rounding boundary may round the other way: one bfloat16 ulp on that
activation.  On test-sized volumes the receptive field of the network covers
the whole volume and a randomly initialised network amplifies such a change:
perturbing every convolution output of the oracle by 1e-7 relative before
its rounding (a handful of flips) moves h = x0 - y by 5e-3 to 6e-3 in
relative L2 norm.  The forward bound is therefore 2^-6 on the relative L2
difference of h and 2^-5 |h|_max on the largest one.  The gradient adds the
GPU's bfloat16 activation gradients (one rounding per stored tensor, about
2^-9 relative) to the same flips: per layer, 2^-5 relative L2.  The
oracle-only test test_parity_tolerance_discriminates shows that a misplaced
tap, a swapped skip connection or transposed channels move the output by
far more than these bounds.
"""
import numpy as np
import pytest

import oracle
from paper_2002_02328_amd import binding, inputs
from gpu_common import rel

pytestmark = pytest.mark.gpu

C, CIN = 16, 1
FWD_REL, FWD_MAX, GRAD_REL = 2.0 ** -6, 2.0 ** -5, 2.0 ** -5


def params(seed, bias=0.02):
    return inputs.net_init_params(seed, C, CIN, head_scale=0.3, bias=bias).astype(np.float32)


def volume(shape, seed, nb=None):
    rng = np.random.default_rng(seed)
    full = shape if nb is None else (nb,) + shape
    return rng.uniform(0.0, 1.0, full).astype(np.float32)


def layer_slices():
    out, off = [], 0
    for co, ci, k in inputs.net_layer_shapes(C, CIN):
        nw = co * ci * k ** 3
        out.append((slice(off, off + nw), slice(off + nw, off + nw + co)))
        off += nw + co
    return out


@pytest.fixture(scope="module")
def net():
    n = binding.Net()
    assert n.num_params == oracle.net_num_params(C, CIN)
    yield n
    n.close()


@pytest.mark.parametrize("shape", [(8, 20, 36), (4, 8, 16), (12, 16, 52)])
def test_forward_matches_oracle(orc, net, shape):
    p = params(11)
    net.set_params(p)
    y = volume(shape, 3)
    x0 = net.forward(y).astype(np.float64)
    ref = oracle.net_forward(p.astype(np.float64), y.astype(np.float64), C, CIN, bf16=True)
    exact = oracle.net_forward(p.astype(np.float64), y.astype(np.float64), C, CIN, bf16=False)
    h_gpu, h_ref, h_exact = x0 - y, ref - y, exact - y
    d = np.linalg.norm(h_gpu - h_ref) / np.linalg.norm(h_ref)
    print("shape %s: |h_gpu - h_bf16| / |h| = %.3e, |h_bf16 - h_fp64| / |h| = %.3e"
          % (shape, d, np.linalg.norm(h_ref - h_exact) / np.linalg.norm(h_ref)))
    assert d <= FWD_REL
    assert np.max(np.abs(h_gpu - h_ref)) <= FWD_MAX * np.max(np.abs(h_ref))


def test_forward_batch_equals_single_volumes(net):
    net.set_params(params(12))
    ys = volume((8, 16, 32), 4, nb=3)
    xb = net.forward(ys)
    for i in range(3):
        assert np.array_equal(xb[i], net.forward(ys[i]))


def test_zero_network_returns_input_exactly(net):
    net.set_params(np.zeros(net.num_params, np.float32))
    y = volume((8, 8, 16), 5)
    assert np.array_equal(net.forward(y), y)


@pytest.mark.parametrize("shape,nb", [((8, 20, 36), 1), ((4, 8, 32), 2)])
def test_gradient_matches_oracle(orc, net, shape, nb):
    p = params(13)
    net.set_params(p)
    y = volume(shape, 6, nb=nb)
    t = (y + 0.1 * np.random.default_rng(7).standard_normal(y.shape)).astype(np.float32)
    loss, g = net.grad(y, t)
    lref, gref = 0.0, np.zeros(p.size)
    for i in range(nb):
        li, gi = oracle.net_loss_grad(p.astype(np.float64), y[i].astype(np.float64),
                                      t[i].astype(np.float64), C, CIN, bf16=True)
        lref += li / nb
        gref += gi / nb
    assert abs(loss - lref) <= 2.0 ** -8 * lref
    for i, (ws, bs) in enumerate(layer_slices()):
        ew, eb = rel(g[ws], gref[ws]), rel(g[bs], gref[bs])
        print("layer %2d: weight grad rel %.2e  bias grad rel %.2e" % (i, ew, eb))
        assert ew <= GRAD_REL, i
        assert eb <= GRAD_REL, i


def test_gradient_is_deterministic(net):
    net.set_params(params(14))
    y = volume((8, 16, 48), 8, nb=2)
    t = volume((8, 16, 48), 9, nb=2)
    l1, g1 = net.grad(y, t)
    l2, g2 = net.grad(y, t)
    assert l1 == l2 and np.array_equal(g1, g2)


def test_adam_first_step(net):
    p = params(15)
    net.set_params(p)
    y = volume((8, 16, 32), 10, nb=2)
    t = volume((8, 16, 32), 11, nb=2)
    loss_g, g = net.grad(y, t)
    lr = 1e-3
    loss = net.train_step(y, t, lr)
    assert loss == loss_g
    step = net.get_params() - p
    # first Adam step: m = (1 - b1) g, v = (1 - b2) g^2, bias-corrected to g and g^2
    expect = -lr * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(step - expect)) <= 1e-3 * lr + 4 * np.spacing(np.abs(p).max())
    # set_params resets the optimiser: the same step again
    net.set_params(p)
    net.train_step(y, t, lr)
    assert np.array_equal(net.get_params() - p, step)


def test_training_reduces_loss(net):
    net.set_params(params(16))
    y = volume((8, 16, 32), 12, nb=2)
    t = np.clip(y * 1.3 - 0.1, 0, 1).astype(np.float32)
    first = net.train_step(y, t, 3e-3)
    for _ in range(30):
        last = net.train_step(y, t, 3e-3)
    assert last < 0.5 * first


def test_save_load_round_trip_and_errors(net):
    p = params(17)
    net.set_params(p)
    blob = net.save()
    assert len(blob) == 24 + 4 * net.num_params
    other = binding.Net()
    other.load(blob)
    assert np.array_equal(other.get_params(), p)
    y = volume((4, 8, 16), 13)
    assert np.array_equal(other.forward(y), net.forward(y))
    with pytest.raises(binding.Bd3mgError):
        other.load(blob[:-4])
    with pytest.raises(binding.Bd3mgError):
        other.load(b"XXXX" + blob[4:])
    with pytest.raises(binding.Bd3mgError):
        other.forward(volume((4, 8, 18), 1))  # sides must be multiples of 4
    bad = p.copy()
    bad[5] = np.nan
    with pytest.raises(binding.Bd3mgError):
        other.set_params(bad)
    other.close()


@pytest.mark.parametrize("prec", [binding.FP32, binding.FP64])
def test_infer_sets_problem_start(net, prec):
    net.set_params(params(18))
    w = inputs.tiny((8, 24, 40), 21, kxy=5, kz=3, nblocks=2)
    nz, ny, nx = w.shape
    g = binding.Problem(nx, ny, nz, prec)
    g.set_psf_gaussian(w.kxy, w.kz, w.sigma_xy, w.sigma_z)
    g.set_params(w.lam, w.delta, w.eta, w.kappa)
    y = (w.xbar + w.noise).astype(g.dtype)
    g.set_data(y)
    g.set_blocks(w.nslices)
    net.infer(g)
    x0 = net.forward(y.astype(np.float32))
    assert np.array_equal(g.get_x(), x0.astype(g.dtype))
    res = g.run(20, check_every=0)
    assert res["sweeps"] == 20 and np.all(np.isfinite(g.get_x()))


def test_full_size_forward_is_translation_consistent(net):
    """256x256x64 volume (the warm start's inference size): the interior of a
    crop aligned to the pooling cells equals the full volume's output there."""
    net.set_params(params(19))
    w = inputs.warmstart_eval_member(0)
    y = (w.xbar + w.noise).astype(np.float32)
    x_full = net.forward(y)
    assert np.all(np.isfinite(x_full))
    z0, y0, x0 = 0, 96, 128
    crop = y[z0:z0 + 64, y0:y0 + 64, x0:x0 + 64]
    x_crop = net.forward(crop)
    m = 24  # beyond the receptive field of the network
    inner = x_crop[m:64 - m, m:64 - m, m:64 - m]
    ref = x_full[z0 + m:z0 + 64 - m, y0 + m:y0 + 64 - m, x0 + m:x0 + 64 - m]
    assert np.array_equal(inner, ref)
