"""Pins of the oracle's three-dimensional total variation: the TV term with
the difference along z inside the root, sum_n sqrt((V^X x)_n^2 + (V^Y x)_n^2
+ (V^Z x)_n^2 + delta^2), the generic ||(D x)_n|| form of the criterion's
regulariser (the paper's criterion, Sec. 3.1, keeps V^Z outside the root as a
separate kappa ||V^Z x||^2; both are options here).

Pinned against closed forms and mathematics, not the oracle's own formulas:
* a volume varying only along z has the closed-form TV value;
* a volume constant along z has the 2D value and gradient;
* the gradient equals central finite differences of f;
* the half-quadratic majorant (omega now with the z difference) majorises f
  on a block and is tangent at the point, for steps along z, in-slice and
  mixed; the block form equals the whole-volume form of a step supported on
  the block (the z difference of the step reaches the slice below it);
* the majorant applied to a block vector agrees with the form;
* BD3MG sweeps decrease f and reach the same minimiser in any block order.
"""
import numpy as np
import pytest


def problem(orc, shape, rng, lam=0.3, delta=0.05, eta=0.4, kappa=0.0, tv3d=True, kz=3):
    nz = shape[0]
    gx = orc.gauss_table(np.linspace(0.6, 1.4, nz), 3)
    gy = orc.gauss_table(np.linspace(0.8, 1.2, nz), 3)
    gz = orc.gauss_table(np.linspace(0.7, 1.5, nz), kz)
    y = rng.uniform(0, 1, size=shape)
    return orc.Problem(y, gx, gy, gz, lam=lam, delta=delta, eta=eta, kappa=kappa, tv3d=tv3d)


def test_closed_form_along_z(orc):
    rng = np.random.default_rng(1)
    shape = (6, 5, 4)
    p = problem(orc, shape, rng)
    a = 0.07
    x = np.broadcast_to(a * np.arange(shape[0])[:, None, None], shape).copy() + 0.2
    t = p.f_terms(x)
    n = shape[1] * shape[2]
    tv = (shape[0] - 1) * n * np.sqrt(a * a + p.delta ** 2) + n * p.delta
    assert abs(t[2] - p.lam * tv) <= 1e-13 * p.lam * tv


def test_constant_along_z_is_the_2d_value(orc):
    rng = np.random.default_rng(2)
    shape = (5, 7, 6)
    p3 = problem(orc, shape, rng, tv3d=True)
    p2 = orc.Problem(p3.y, p3.gx, p3.gy, p3.gz, lam=p3.lam, delta=p3.delta, eta=p3.eta, tv3d=False)
    x = np.broadcast_to(rng.uniform(0, 1, size=shape[1:]), shape).copy()
    assert p3.f_terms(x)[2] == p2.f_terms(x)[2]
    assert np.allclose(p3.grad(x), p2.grad(x), rtol=0, atol=1e-15)
    # and with a z ramp the two differ
    x[2:] += 0.3
    assert p3.f_terms(x)[2] > p2.f_terms(x)[2]


@pytest.mark.parametrize("kappa", [0.0, 0.2])
def test_gradient_finite_differences(orc, kappa):
    rng = np.random.default_rng(3)
    shape = (6, 7, 8)
    p = problem(orc, shape, rng, lam=0.05, delta=0.1, eta=0.7, kappa=kappa)
    x = rng.uniform(0.1, 0.9, size=shape)
    g = p.grad(x)
    for _ in range(6):
        v = rng.standard_normal(shape)
        v /= np.linalg.norm(v)
        eps = 1e-5
        fd = (p.f(x + eps * v) - p.f(x - eps * v)) / (2 * eps)
        assert abs(fd - float((g * v).sum())) <= 1e-7 * max(1.0, np.linalg.norm(g))


def test_majorant_inequality_and_tangency(orc):
    rng = np.random.default_rng(4)
    shape = (7, 6, 5)
    for trial in range(45):
        p = problem(orc, shape, rng, lam=0.4, delta=0.03, eta=0.0 if trial % 2 else 0.5)
        x = rng.uniform(-0.2, 1.2, size=shape)
        z0 = int(rng.integers(0, 6))
        n = int(rng.integers(1, 7 - z0 + 1))
        v = np.zeros(shape)
        kind = trial % 3  # along z only, in-slice only, mixed
        base = rng.standard_normal((n,) + shape[1:])
        if kind == 0:
            base = np.broadcast_to(rng.standard_normal((n, 1, 1)), base.shape)
        elif kind == 1:
            base = base - base.mean(axis=0, keepdims=True)
        v[z0:z0 + n] = [0.02, 0.4, 3.0][trial % 3] * base
        f0, g = p.f(x), p.grad(x)
        q = f0 + float((g * v).sum()) + 0.5 * p.majorant_form(x, v, v, z0, z0 + n)
        assert p.f(x + v) <= q + 1e-12 * max(1.0, abs(q)), trial
        # the block form of a step supported on the block is its whole-volume form
        full = p.majorant_form(x, v, v, 0, shape[0])
        assert abs(p.majorant_form(x, v, v, z0, z0 + n) - full) <= 1e-12 * abs(full)
        gaps = []
        for t in (1e-2, 5e-3):
            qt = f0 + t * float((g * v).sum()) + 0.5 * t * t * p.majorant_form(x, v, v, z0, z0 + n)
            gaps.append(qt - p.f(x + t * v))
        assert gaps[1] <= 0.3 * gaps[0] + 1e-11


def test_majorant_apply_agrees_with_the_form(orc):
    rng = np.random.default_rng(5)
    shape = (7, 8, 6)
    p = problem(orc, shape, rng, kappa=0.05, kz=5)
    x = rng.uniform(-0.2, 1.2, size=shape)
    for z0, z1 in [(0, 2), (2, 5), (4, 7)]:
        u = np.zeros(shape)
        w = np.zeros(shape)
        u[z0:z1] = rng.standard_normal((z1 - z0,) + shape[1:])
        w[z0:z1] = rng.standard_normal((z1 - z0,) + shape[1:])
        au = p.majorant_apply(x, u, z0, z1)
        form = p.majorant_form(x, u, w, z0, z1)
        assert abs(float((w * au).sum()) - form) <= 1e-12 * abs(form)


def test_sweeps_decrease_f_and_agree_on_the_minimiser(orc):
    rng = np.random.default_rng(6)
    shape = (8, 9, 10)
    p = problem(orc, shape, rng, lam=0.05, delta=0.05, eta=0.3)
    nsl = [3, 2, 3]
    xs = []
    for order in ([0, 1, 2], [2, 0, 1]):
        x = p.y.copy()
        d = np.zeros(shape)
        fs = [p.f(x)]
        for _ in range(40):
            p.run(x, d, nsl, order, 1, history=False)
            fs.append(p.f(x))
        assert all(b <= a + 1e-13 * abs(a) for a, b in zip(fs, fs[1:]))
        p.run(x, d, nsl, order, 1500, history=False)
        xs.append(x)
    assert np.linalg.norm(xs[0] - xs[1]) <= 1e-7 * np.linalg.norm(xs[0])


def test_lipschitz_bound_covers_the_z_difference(orc):
    """With no blur, box or z penalty the curvature of f at a flat volume is
    lambda / delta V^T V; on the 3D checkerboard v = (-1)^(i+j+k) its Rayleigh
    quotient is 4 times the share of forward differences per voxel along each
    axis (10.33 on 6x8x8), above the 8 of the in-slice operators alone, so
    the bound must take 12 lambda / delta (each forward difference has norm at
    most 2)."""
    shape = (6, 8, 8)
    nz, ny, nx = shape
    lam, delta = 0.3, 0.05
    zero = np.zeros((nz, 3))
    p = orc.Problem(np.zeros(shape), zero, zero, np.zeros((nz, 3)), lam=lam, delta=delta, tv3d=True)
    k, j, i = np.indices(shape)
    v = (-1.0) ** (i + j + k)
    x = np.full(shape, 0.5)
    t = 1e-6 * delta
    q = float((v * (p.grad(x + t * v) - p.grad(x))).sum() / (t * (v * v).sum()))
    share = ((nx - 1) * ny * nz + nx * (ny - 1) * nz + nx * ny * (nz - 1)) / (nx * ny * nz)
    assert abs(q - 4 * share * lam / delta) <= 1e-6 * q
    L = p.lipschitz_bound()
    assert abs(L - 12 * lam / delta) <= 1e-12 * L
    assert 8 * lam / delta < q <= L
    p2 = orc.Problem(np.zeros(shape), zero, zero, np.zeros((nz, 3)), lam=lam, delta=delta)
    assert abs(p2.lipschitz_bound() - 8 * lam / delta) <= 1e-12 * L
