"""Pins of the oracle's general per-depth kernels (the rotated Gaussian blur
of the paper's experiments, Sec. 3.1: a kernel of its own variance and
rotation at every depth), each against a fact that does not come from the
oracle's general path itself:

* a kernel that is the tensor product gz_k (x) gy_k (x) gx_k gives the
  separable operator (pinned in test_oracle_pins);
* a single tap at (c, b, a) shifts the volume by (c, b, a) and the kernel of
  an output slice is its own (a point source's image in output slice k is
  P_k read at k - s);
* <Hx, r> = <x, H^T r> for random kernels that differ per slice;
* the rotated Gaussian at rotation 0 is the product of the three normalised
  1-D Gaussians, at pi / 2 its in-slice transpose, and at any angle centrally
  symmetric with unit sum;
* grad f matches central differences, the Lipschitz bound bounds ||H^T H||
  from above, and the block MM steps decrease f.
"""
import numpy as np
import pytest

import oracle
from paper_2002_02328_amd import inputs

pytestmark = pytest.mark.filterwarnings("ignore")


def rnd(shape, seed):
    return np.random.default_rng(seed).random(shape)


def test_tensor_product_kernels_equal_separable_operator(orc):
    nz, ny, nx = 6, 11, 13
    rng = np.random.default_rng(1)
    gx, gy, gz = rng.random((nz, 5)), rng.random((nz, 3)), rng.random((nz, 5))
    pk = np.einsum("kc,kb,ka->kcba", gz, gy, gx)
    y = rnd((nz, ny, nx), 2)
    sep = oracle.Problem(y, gx, gy, gz)
    gen = oracle.Problem.with_kernels(y, pk)
    x, r = rnd((nz, ny, nx), 3), rnd((nz, ny, nx), 4)
    assert np.allclose(gen.H(x), sep.H(x), rtol=1e-13, atol=1e-13)
    assert np.allclose(gen.HT(r), sep.HT(r), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("tap", [(1, -2, 1), (-2, 0, -1), (0, 1, 2)])
def test_single_tap_shifts_the_volume(orc, tap):
    nz, ny, nx = 7, 9, 10
    kz, ky, kx = 5, 5, 5
    c, b, a = tap
    pk = np.zeros((nz, kz, ky, kx))
    pk[:, c + 2, b + 2, a + 2] = 1.0
    x = rnd((nz, ny, nx), 5)
    o = oracle.Problem.with_kernels(np.zeros_like(x), pk)
    want = np.zeros_like(x)
    # (Hx)_{k,j,i} = x_{k-c, j-b, i-a}, zero outside the volume
    ks, js, is_ = slice(max(c, 0), nz + min(c, 0)), slice(max(b, 0), ny + min(b, 0)), slice(max(a, 0), nx + min(a, 0))
    kd, jd, id_ = slice(max(-c, 0), nz - max(c, 0)), slice(max(-b, 0), ny - max(b, 0)), slice(max(-a, 0), nx - max(a, 0))
    want[ks, js, is_] = x[kd, jd, id_]
    assert np.array_equal(o.H(x), want)


def test_point_source_reads_the_output_slice_kernel(orc):
    nz, ny, nx, kz, kxy = 7, 9, 9, 5, 3
    pk = rnd((nz, kz, kxy, kxy), 6)
    x = np.zeros((nz, ny, nx))
    s, j0, i0 = 3, 4, 4
    x[s, j0, i0] = 1.0
    hx = oracle.Problem.with_kernels(np.zeros_like(x), pk).H(x)
    for k in range(nz):
        c = k - s
        if abs(c) > kz // 2:
            assert not hx[k].any()
            continue
        assert np.array_equal(hx[k, j0 - 1:j0 + 2, i0 - 1:i0 + 2], pk[k, c + kz // 2])


def test_adjoint_identity_with_depth_variant_kernels(orc):
    nz, ny, nx = 8, 12, 10
    pk = rnd((nz, 7, 5, 3), 7) - 0.3
    o = oracle.Problem.with_kernels(np.zeros((nz, ny, nx)), pk)
    x, r = rnd((nz, ny, nx), 8), rnd((nz, ny, nx), 9)
    lhs, rhs = np.vdot(o.H(x), r), np.vdot(x, o.HT(r))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_rotated_gaussian_special_angles(orc):
    nz, kxy, kz = 4, 7, 5
    rng = np.random.default_rng(10)
    sx, sy, sz = rng.uniform(0.5, 2, nz), rng.uniform(0.5, 2, nz), rng.uniform(0.7, 2, nz)
    p0 = oracle.rotated_gauss_kernels(sx, sy, np.zeros(nz), sz, kxy, kz)
    sep = np.einsum("kc,kb,ka->kcba", oracle.gauss_table(sz, kz), oracle.gauss_table(sy, kxy),
                    oracle.gauss_table(sx, kxy))
    assert np.allclose(p0, sep, rtol=1e-13, atol=1e-16)
    p90 = oracle.rotated_gauss_kernels(sx, sy, np.full(nz, np.pi / 2), sz, kxy, kz)
    assert np.allclose(p90, np.swapaxes(sep, 2, 3), rtol=1e-12, atol=1e-15)
    th = rng.uniform(0, np.pi, nz)
    pt = oracle.rotated_gauss_kernels(sx, sy, th, sz, kxy, kz)
    assert np.allclose(pt.sum(axis=(1, 2, 3)), 1.0, rtol=1e-14)
    assert np.allclose(pt, pt[:, ::-1, ::-1, ::-1], rtol=1e-13, atol=1e-17)
    # rotating by theta + pi gives the same kernel; generic angles are not separable
    assert np.allclose(oracle.rotated_gauss_kernels(sx, sy, th + np.pi, sz, kxy, kz), pt, rtol=1e-12, atol=1e-16)
    m = pt[0, kz // 2]
    assert np.linalg.matrix_rank(m, tol=1e-10 * m.max()) > 1
    # rotation by +pi/4 of a kernel long along its first axis: long along the
    # diagonal a = b (index order [c][b][a])
    q = oracle.rotated_gauss_kernels([2.0], [0.5], [np.pi / 4], [1.0], kxy, kz)[0, kz // 2]
    r = kxy // 2
    assert q[r + 1, r + 1] > 10 * q[r - 1, r + 1] and q[r - 1, r - 1] > 10 * q[r + 1, r - 1]


def _dense_problem(shape, seed, **kw):
    w = inputs.tiny_dense(shape, seed, **kw)
    ps = w.extra["psf"]
    pk = oracle.rotated_gauss_kernels(ps["sx"], ps["sy"], ps["theta"], ps["sz"], w.kxy, w.kz)
    y = oracle.Problem.with_kernels(np.zeros(shape), pk).H(w.xbar) + w.noise
    o = oracle.Problem.with_kernels(y, pk, lam=w.lam, delta=w.delta, eta=w.eta, kappa=w.kappa)
    return w, pk, y, o


def test_gradient_matches_central_differences(orc):
    w, pk, y, o = _dense_problem((5, 8, 9), 11, kxy=5, kz=3, kappa=0.05)
    x = y + 0.1 * rnd(y.shape, 12)
    g = o.grad(x)
    rng = np.random.default_rng(13)
    for _ in range(6):
        v = (rng.integers(0, 5), rng.integers(0, 8), rng.integers(0, 9))
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[v] += h
        xm[v] -= h
        fd = (o.f(xp) - o.f(xm)) / (2 * h)
        assert abs(fd - g[v]) <= 1e-6 * max(1.0, abs(g[v]))


def test_lipschitz_bound_bounds_the_data_term(orc):
    nz, ny, nx = 6, 16, 16
    pk = oracle.rotated_gauss_kernels(*[np.random.default_rng(14).uniform(0.5, 2, nz) for _ in range(2)],
                                      np.random.default_rng(15).uniform(0, np.pi, nz),
                                      np.random.default_rng(16).uniform(0.6, 2, nz), 5, 5)
    o = oracle.Problem.with_kernels(np.zeros((nz, ny, nx)), pk, lam=0.0, delta=1.0, eta=0.0)
    v = rnd((nz, ny, nx), 17)
    for _ in range(60):
        v = o.HT(o.H(v))
        v /= np.linalg.norm(v)
    est = np.linalg.norm(o.HT(o.H(v)))
    L = o.lipschitz_bound()
    assert est <= L <= 2.0 * est


def test_block_steps_decrease_f(orc):
    w, pk, y, o = _dense_problem((8, 12, 14), 18, kxy=5, kz=5)
    x, d = y.copy(), np.zeros(y.shape)
    order = np.arange(len(w.nslices), dtype=np.int32)
    prev = o.f(x)
    for _ in range(5):
        o.run(x, d, w.nslices, order, 1, history=False)
        f = o.f(x)
        assert f <= prev * (1 + 1e-14)
        prev = f
