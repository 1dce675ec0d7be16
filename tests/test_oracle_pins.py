"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed
forms, a library routine (scipy's convolution, numpy's pseudo-inverse and
linear solve), textbook conjugate gradients, brute-force matrices, finite
differences, or the invariants the paper states (majorisation, Sec. 2.2;
monotone decrease without delays, Sec. 2.4).
"""
import numpy as np
import pytest
import scipy.ndimage

from paper_2002_02328_amd import inputs


def rand_tables(rng, nz, k, positive=True):
    """Asymmetric per-slice tables (not Gaussian) so that transposes show."""
    t = rng.uniform(0.1, 1.0, size=(nz, k)) if positive else rng.standard_normal((nz, k))
    return t


def make_problem(orc, shape, rng, kx=3, ky=5, kz=3, dense=False, lam=0.0, delta=0.1, eta=0.0,
                 kappa=0.0, tables=None, y=None):
    nz, ny, nx = shape
    if tables is None:
        gx, gy, gz = rand_tables(rng, nz, kx), rand_tables(rng, nz, ky), rand_tables(rng, nz, kz)
    else:
        gx, gy, gz = tables
    if y is None:
        y = rng.uniform(0, 1, size=shape)
    return orc.Problem(y, gx, gy, gz, lam=lam, delta=delta, eta=eta, kappa=kappa, dense=dense)


# ---------------------------------------------------------------- PSF tables

def test_gauss_table_normalised_and_gaussian(orc):
    sig = np.array([0.5, 0.9, 1.7, 3.0])
    k = 9
    t = orc.gauss_table(sig, k)
    assert np.allclose(t.sum(axis=1), 1.0, atol=1e-15)
    r = k // 2
    assert np.allclose(t, t[:, ::-1], rtol=0, atol=0)  # symmetric
    # log of consecutive ratios: log(g[a+1]/g[a]) = -(2a+1) / (2 sigma^2)
    for z, s in enumerate(sig):
        a = np.arange(-r, r)
        lr = np.log(t[z, 1:] / t[z, :-1])
        assert np.allclose(lr, -(2 * a + 1) / (2 * s * s), rtol=1e-12, atol=1e-12)


def test_gauss_table_second_moment(orc):
    # A wide, untruncated discrete Gaussian has variance sigma^2 up to a Poisson
    # summation error of order sigma^4 exp(-2 pi^2 sigma^2), negligible for sigma >= 1.5.
    for s in (1.5, 2.0, 2.5):
        t = orc.gauss_table([s], 41)[0]
        a = np.arange(-20, 21)
        assert abs((t * a * a).sum() - s * s) < 1e-8


# ---------------------------------------------------------------- H and H^T

@pytest.mark.parametrize("dense", [True, False])
def test_adjoint_identity(orc, dense):
    rng = np.random.default_rng(1)
    for shape, ks in [((5, 6, 7), (3, 5, 3)), ((7, 9, 8), (5, 3, 5)), ((3, 4, 11), (1, 3, 7))]:
        p = make_problem(orc, shape, rng, *ks, dense=dense)
        x = rng.standard_normal(shape)
        r = rng.standard_normal(shape)
        hx, htr = p.H(x), p.HT(r)
        lhs, rhs = float((hx * r).sum()), float((x * htr).sum())
        assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(hx) * np.linalg.norm(r)


def test_dense_equals_separable(orc):
    rng = np.random.default_rng(2)
    shape = (6, 7, 9)
    tabs = (rand_tables(rng, 6, 5), rand_tables(rng, 6, 3), rand_tables(rng, 6, 5))
    y = rng.uniform(size=shape)
    pd = make_problem(orc, shape, rng, tables=tabs, y=y, dense=True)
    ps = make_problem(orc, shape, rng, tables=tabs, y=y, dense=False)
    x = rng.standard_normal(shape)
    for a, b in [(pd.H(x), ps.H(x)), (pd.HT(x), ps.HT(x))]:
        assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(a))


@pytest.mark.parametrize("dense", [True, False])
def test_depth_invariant_equals_scipy_convolve(orc, dense):
    rng = np.random.default_rng(3)
    shape = (6, 8, 10)
    gx1, gy1, gz1 = rng.uniform(0.1, 1, 5), rng.uniform(0.1, 1, 3), rng.uniform(0.1, 1, 3)
    tabs = (np.tile(gx1, (6, 1)), np.tile(gy1, (6, 1)), np.tile(gz1, (6, 1)))
    p = make_problem(orc, shape, rng, tables=tabs, dense=dense)
    w = gz1[:, None, None] * gy1[None, :, None] * gx1[None, None, :]
    x = rng.standard_normal(shape)
    ref = scipy.ndimage.convolve(x, w, mode="constant", cval=0.0)
    assert np.allclose(p.H(x), ref, rtol=0, atol=1e-13)
    # adjoint of a convolution is the correlation with the same kernel
    ref_t = scipy.ndimage.correlate(x, w, mode="constant", cval=0.0)
    assert np.allclose(p.HT(x), ref_t, rtol=0, atol=1e-13)


def dense_matrix(op, shape):
    n = int(np.prod(shape))
    M = np.zeros((n, n))
    for q in range(n):
        e = np.zeros(n)
        e[q] = 1.0
        M[:, q] = op(e.reshape(shape)).ravel()
    return M


def test_brute_force_matrix_transpose(orc):
    rng = np.random.default_rng(4)
    shape = (4, 3, 5)
    p = make_problem(orc, shape, rng, 3, 3, 3, dense=True)
    M = dense_matrix(p.H, shape)
    MT = dense_matrix(p.HT, shape)
    assert np.array_equal(MT, M.T)
    ps = make_problem(orc, shape, rng, tables=(p.gx, p.gy, p.gz), dense=False)
    assert np.allclose(dense_matrix(ps.H, shape), M, rtol=1e-15, atol=1e-16)


def test_impulse_response_uses_output_slice_kernel(orc):
    # Output-slice indexing: the response to an impulse at depth k0, seen at
    # output depth k, is gz_k[k-k0] * gy_k (x) gx_k -- the factors of slice k.
    rng = np.random.default_rng(5)
    shape = (5, 9, 9)
    p = make_problem(orc, shape, rng, 3, 3, 3, dense=False)
    x = np.zeros(shape)
    k0, j0, i0 = 2, 4, 4
    x[k0, j0, i0] = 1.0
    h = p.H(x)
    for k in (1, 2, 3):
        prof = np.zeros((9, 9))
        prof[3:6, 3:6] = np.outer(p.gy[k], p.gx[k]) * p.gz[k, k - k0 + 1]
        assert np.allclose(h[k], prof, rtol=1e-15, atol=1e-17)
    assert np.all(h[0] == 0) and np.all(h[4] == 0)


def test_unit_dc_gain_interior(orc):
    rng = np.random.default_rng(6)
    shape = (9, 12, 13)
    sig = rng.uniform(0.4, 2.0, size=9)
    t5 = orc.gauss_table(sig, 5)
    tz = orc.gauss_table(rng.uniform(0.5, 1.5, size=9), 3)
    for dense in (True, False):
        p = make_problem(orc, shape, rng, tables=(t5, t5, tz), dense=dense)
        h = p.H(np.ones(shape))
        assert np.allclose(h[1:-1, 2:-2, 2:-2], 1.0, rtol=0, atol=1e-14)
        assert np.all(h[0] < 1.0)  # missing slice beyond the volume


# ------------------------------------------------------------ V operators

def test_difference_operators(orc):
    rng = np.random.default_rng(7)
    shape = (4, 5, 6)
    p = make_problem(orc, shape, rng)
    k, j, i = np.meshgrid(np.arange(4), np.arange(5), np.arange(6), indexing="ij")
    ramp = 2.0 * i + 3.0 * j - 5.0 * k
    vx, vy, vz = p.V(ramp, "x"), p.V(ramp, "y"), p.V(ramp, "z")
    assert np.all(vx[:, :, :-1] == 2.0) and np.all(vx[:, :, -1] == 0.0)
    assert np.all(vy[:, :-1, :] == 3.0) and np.all(vy[:, -1, :] == 0.0)
    assert np.all(vz[:-1] == -5.0) and np.all(vz[-1] == 0.0)
    for ax in "xyz":
        M = dense_matrix(lambda v: p.V(v, ax), shape)
        MT = dense_matrix(lambda v: p.V(v, ax, adjoint=True), shape)
        assert np.array_equal(MT, M.T)


# -------------------------------------------------------------- criterion

def identity_tables(nz):
    one = np.ones((nz, 1))
    return one, one, one


def test_f_closed_forms(orc):
    shape = (3, 4, 5)
    N = 60
    rng = np.random.default_rng(8)
    y = rng.uniform(size=shape)
    lam, delta, eta, kappa = 0.3, 0.07, 0.9, 0.4
    p = orc.Problem(y, *identity_tables(3), lam=lam, delta=delta, eta=eta, kappa=kappa)
    # constant volume inside the box: TV = lambda N delta, box = 0, V^Z = 0
    c = 0.37
    t = p.f_terms(np.full(shape, c))
    assert np.isclose(t[0], 0.5 * ((c - y) ** 2).sum(), rtol=1e-14)
    assert t[1] == 0.0 and t[3] == 0.0
    assert np.isclose(t[2], lam * N * delta, rtol=1e-14)
    # values outside the box: eta * sum of squared distances to [0, 1]
    x = rng.uniform(-1, 2, size=shape)
    dist = np.maximum(0, x - 1) + np.maximum(0, -x)
    assert np.isclose(p.f_terms(x)[1], eta * (dist ** 2).sum(), rtol=1e-14)
    # ramp along z: kappa * sum of squared z-differences
    k = np.arange(3)[:, None, None] * np.ones(shape)
    assert np.isclose(p.f_terms(0.1 * k)[3], kappa * 0.01 * (2 * 4 * 5), rtol=1e-12)
    # ramp along x: each voxel with a difference of 0.1 in x, 0 in y
    i = np.arange(5)[None, None, :] * np.ones(shape)
    tv = lam * (3 * 4 * (4 * np.sqrt(0.01 + delta ** 2) + delta))
    assert np.isclose(p.f_terms(0.1 * i)[2], tv, rtol=1e-13)


@pytest.mark.parametrize("dense", [True, False])
def test_gradient_finite_differences(orc, dense):
    rng = np.random.default_rng(9)
    shape = (6, 7, 8)
    for kappa in (0.0, 0.3):
        p = make_problem(orc, shape, rng, 3, 3, 3, dense=dense, lam=0.05, delta=0.1, eta=0.7,
                         kappa=kappa)
        # keep clear of the box kinks at 0 and 1: values in (0.1, 0.9) or well outside
        x = rng.uniform(0.1, 0.9, size=shape)
        mask = rng.uniform(size=shape)
        x[mask < 0.15] = rng.uniform(1.2, 1.5, size=int((mask < 0.15).sum()))
        x[mask > 0.85] = rng.uniform(-0.5, -0.2, size=int((mask > 0.85).sum()))
        g = p.grad(x)
        for _ in range(5):
            v = rng.standard_normal(shape)
            v /= np.linalg.norm(v)
            eps = 1e-5
            fd = (p.f(x + eps * v) - p.f(x - eps * v)) / (2 * eps)
            an = float((g * v).sum())
            assert abs(fd - an) <= 1e-7 * max(1.0, np.linalg.norm(g))


def test_gradient_slices_match_full(orc):
    rng = np.random.default_rng(10)
    shape = (9, 6, 7)
    p = make_problem(orc, shape, rng, 3, 3, 5, lam=0.05, delta=0.1, eta=0.7, kappa=0.2)
    x = rng.uniform(-0.2, 1.2, size=shape)
    g = p.grad(x)
    gs = p.grad(x, 3, 6)
    assert np.array_equal(gs[3:6], g[3:6])
    assert np.all(gs[:3] == 0) and np.all(gs[6:] == 0)


# ---------------------------------------------------------------- majorant

@pytest.mark.parametrize("dense", [True, False])
def test_majorant_inequality_and_tangency(orc, dense):
    # Sec. 2.2: Q_S(v; x~) >= f on block S with equality at v = 0; the
    # half-quadratic matrix must satisfy it for any step, box crossings included.
    rng = np.random.default_rng(11)
    shape = (8, 6, 7)
    worst = -np.inf
    for trial in range(60):
        kappa = 0.0 if trial % 2 else 0.25
        p = make_problem(orc, shape, rng, 3, 3, 3, dense=dense, lam=0.08, delta=0.05, eta=0.6,
                         kappa=kappa)
        x = rng.uniform(-0.3, 1.3, size=shape)
        z0 = int(rng.integers(0, 7))
        n = int(rng.integers(1, 8 - z0 + 1))
        v = np.zeros(shape)
        scale = [0.01, 0.3, 3.0][trial % 3]
        v[z0:z0 + n] = scale * rng.standard_normal((n,) + shape[1:])
        f0 = p.f(x)
        g = p.grad(x)
        q = f0 + float((g * v).sum()) + 0.5 * p.majorant_form(x, v, v, z0, z0 + n)
        fv = p.f(x + v)
        worst = max(worst, (fv - q) / max(1.0, abs(q)))
        assert fv <= q + 1e-12 * max(1.0, abs(q))
        # tangency: the gap vanishes to second order as the step shrinks
        gaps = []
        for t in (1e-2, 5e-3):
            qt = f0 + t * float((g * v).sum()) + 0.5 * t * t * p.majorant_form(x, v, v, z0, z0 + n)
            gaps.append(qt - p.f(x + t * v))
        assert gaps[1] <= 0.3 * gaps[0] + 1e-11
    assert worst <= 0


def test_majorant_inequality_tv_curvature(orc):
    # eta = kappa = 0 isolates the total-variation curvature: the data term is
    # exactly quadratic, so any missing part of lambda D^T Diag(omega) D shows as
    # Q < f for steps that change the x- or y-differences.
    rng = np.random.default_rng(15)
    shape = (4, 9, 10)
    for trial in range(40):
        p = make_problem(orc, shape, rng, 3, 3, 3, lam=0.5, delta=0.02, eta=0.0, kappa=0.0)
        x = rng.uniform(0, 1, size=shape)
        z0 = int(rng.integers(0, 4))
        v = np.zeros(shape)
        axis = trial % 3  # vary along y only, along x only, or both
        base = rng.standard_normal(shape[1:])
        if axis == 0:
            base = np.repeat(base[:, :1], shape[2], axis=1)
        elif axis == 1:
            base = np.repeat(base[:1, :], shape[1], axis=0)
        v[z0] = [0.05, 0.5, 2.0][trial % 3 if trial < 20 else 2] * base
        q = p.f(x) + float((p.grad(x) * v).sum()) + 0.5 * p.majorant_form(x, v, v, z0, z0 + 1)
        assert p.f(x + v) <= q + 1e-12 * abs(q)


def test_majorant_exact_for_quadratic_part(orc):
    # with lambda = 0 and the iterate and step inside the box, f is exactly quadratic
    # with Hessian H^T H + 2 kappa V^Z^T V^Z, so Q equals f.
    rng = np.random.default_rng(12)
    shape = (6, 5, 6)
    p = make_problem(orc, shape, rng, 3, 3, 3, lam=0.0, eta=0.5, kappa=0.3)
    x = rng.uniform(0.3, 0.7, size=shape)
    v = np.zeros(shape)
    v[2:4] = 0.1 * rng.uniform(-1, 1, size=(2,) + shape[1:])
    q = p.f(x) + float((p.grad(x) * v).sum()) + 0.5 * (p.majorant_form(x, v, v, 2, 4)
                                                        - 2 * 0.5 * float((v * v).sum()))
    assert np.isclose(p.f(x + v), q, rtol=1e-12)


def test_majorant_form_symmetric_bilinear(orc):
    rng = np.random.default_rng(13)
    shape = (6, 5, 6)
    p = make_problem(orc, shape, rng, 3, 3, 3, lam=0.1, eta=0.5, kappa=0.3, delta=0.05)
    x = rng.uniform(size=shape)
    u, v, w = (rng.standard_normal(shape) for _ in range(3))
    a = p.majorant_form
    assert np.isclose(a(x, u, v), a(x, v, u), rtol=1e-13)
    assert np.isclose(a(x, u, 2 * v + w), 2 * a(x, u, v) + a(x, u, w), rtol=1e-12)
    assert a(x, u, u) > 0


# ----------------------------------------------------------- 2x2 pinv

def test_pinv2_matches_numpy(orc):
    rng = np.random.default_rng(14)
    for _ in range(200):
        A = rng.standard_normal((2, 2))
        B = A @ A.T
        P = orc.pinv2(B[0, 0], B[0, 1], B[1, 1])
        assert np.allclose(P, np.linalg.pinv(B), rtol=1e-9, atol=1e-12)
    for _ in range(200):
        v = rng.standard_normal(2) * 10.0 ** rng.uniform(-3, 3)
        B = np.outer(v, v)
        P = orc.pinv2(B[0, 0], B[0, 1], B[1, 1])
        assert np.allclose(P, np.linalg.pinv(B), rtol=1e-9, atol=1e-12 * np.abs(P).max())
    for b11 in (2.0, 1e-30):
        P = orc.pinv2(b11, 0.0, 0.0)  # second direction zero (first visit)
        assert np.allclose(P, [[1 / b11, 0], [0, 0]], rtol=1e-14)
    assert np.all(orc.pinv2(0.0, 0.0, 0.0) == 0)


# ------------------------------------------------------------ worker step

def tiny_problem(orc, shape=(8, 9, 10), seed=20, lam=0.02, delta=0.05, eta=0.3, kappa=0.0,
                 kxy=3, kz=3, dense=False):
    w = inputs.tiny(shape, seed, kxy=kxy, kz=kz, lam=lam, delta=delta, eta=eta, kappa=kappa)
    gx = orc.gauss_table(w.sigma_xy, kxy)
    gz = orc.gauss_table(w.sigma_z, kz)
    p0 = orc.Problem(np.zeros(shape), gx, gx, gz, dense=dense)
    y = p0.H(w.xbar) + w.noise
    return orc.Problem(y, gx, gx, gz, lam=lam, delta=delta, eta=eta, kappa=kappa, dense=dense), w


def test_first_visit_is_majorised_steepest_descent(orc):
    p, w = tiny_problem(orc)
    x = p.y.copy()
    dprev = np.zeros(p.shape)
    g = p.grad(x)
    gS = np.zeros(p.shape)
    gS[2:5] = g[2:5]
    step = (gS * gS).sum() / p.majorant_form(x, gS, gS, 2, 5)
    x_ref = x - step * gS
    info = p.block_step(x, dprev, 2, 3)
    assert np.allclose(x, x_ref, rtol=1e-13, atol=1e-15)
    assert np.allclose(dprev, -step * gS, rtol=1e-13, atol=1e-15)
    assert info[6] == 0.0


def test_bd3mg_single_block_equals_textbook_cg(orc):
    # B = 1 and lambda = eta = kappa = 0: f = 1/2 ||Hx - y||^2 and the majorant is f
    # itself, so the memory-gradient subspace step reproduces conjugate gradients
    # on H^T H x = H^T y (each CG iterate minimises f over x_k + span{r_k, p_{k-1}}).
    rng = np.random.default_rng(21)
    shape = (4, 5, 6)
    tabs = (orc.gauss_table(rng.uniform(0.5, 1.2, 4), 3), orc.gauss_table(rng.uniform(0.5, 1.2, 4), 3),
            orc.gauss_table(rng.uniform(0.5, 1.0, 4), 3))
    y = rng.uniform(size=shape)
    p = orc.Problem(y, *tabs, lam=0.0, delta=1.0, eta=0.0)
    M = dense_matrix(p.H, shape)
    A = M.T @ M
    b = M.T @ y.ravel()
    xc = y.ravel().copy()
    r = b - A @ xc
    pdir = r.copy()
    x = y.copy()
    dprev = np.zeros(shape)
    # rounding differences between the two recurrences grow with the iteration
    # count; ten iterations already expose any error in the subspace step.
    for it in range(10):
        Ap = A @ pdir
        alpha = (r @ r) / (pdir @ Ap)
        xc = xc + alpha * pdir
        rn = r - alpha * Ap
        beta = (rn @ rn) / (r @ r)
        pdir = rn + beta * pdir
        r = rn
        p.block_step(x, dprev, 0, shape[0])
        assert np.linalg.norm(x.ravel() - xc) <= 1e-10 * np.linalg.norm(xc), it


@pytest.mark.parametrize("order_kind", ["natural", "colored"])
def test_limit_is_normal_equations_solution(orc, order_kind):
    rng = np.random.default_rng(22)
    shape = (6, 4, 5)
    tabs = (orc.gauss_table(np.full(6, 0.5), 3), orc.gauss_table(np.full(6, 0.6), 3),
            orc.gauss_table(np.full(6, 0.7), 3))
    y = rng.uniform(size=shape)
    p = orc.Problem(y, *tabs, lam=0.0, delta=1.0, eta=0.0)
    M = dense_matrix(p.H, shape)
    xs = np.linalg.solve(M.T @ M, M.T @ y.ravel())
    nsl = [2, 1, 3]
    if order_kind == "natural":
        order = [0, 1, 2]
    else:
        _, order, _ = orc.color_schedule(nsl, 2 * p.rz)
    x = y.copy()
    dprev = np.zeros(shape)
    p.run(x, dprev, nsl, order, 400, history=False)
    assert np.linalg.norm(x.ravel() - xs) <= 1e-9 * np.linalg.norm(xs)


def test_monotone_decrease_each_block_update(orc):
    # Sec. 2.4: without delays every block update decreases f.
    p, w = tiny_problem(orc, shape=(9, 10, 11), lam=0.03, delta=0.02, eta=0.5, kappa=0.1)
    x = p.y.copy() * 1.3 - 0.1  # start partly outside the box
    dprev = np.zeros(p.shape)
    nsl = [2, 3, 1, 3]
    z0 = np.concatenate([[0], np.cumsum(nsl)[:-1]])
    f = p.f(x)
    for sweep in range(6):
        for b in range(4):
            p.block_step(x, dprev, int(z0[b]), nsl[b])
            fn = p.f(x)
            assert fn <= f + 1e-13 * abs(f)
            f = fn


# --------------------------------------------------------------- schedule

def test_coloring_valid_and_greedy(orc):
    rng = np.random.default_rng(23)
    for _ in range(50):
        nb = int(rng.integers(1, 20))
        nsl = rng.integers(1, 7, size=nb)
        gap = int(rng.integers(0, 9))
        nc, order, color = orc.color_schedule(nsl, gap)
        z0 = np.concatenate([[0], np.cumsum(nsl)[:-1]])
        assert sorted(order.tolist()) == list(range(nb))
        assert color.max() + 1 == nc
        # colour-major, z ascending within a colour
        keys = [(color[b], z0[b]) for b in order]
        assert keys == sorted(keys)
        for a in range(nb):
            for b in range(a + 1, nb):
                if color[a] == color[b]:
                    assert z0[b] - (z0[a] + nsl[a]) >= gap
            # greedy: every smaller colour has an earlier block too close
            for c in range(color[a]):
                assert any(color[e] == c and z0[a] - (z0[e] + nsl[e]) < gap for e in range(a))


def test_same_color_blocks_commute_exactly(orc):
    # Blocks at least 2 r_z slices apart read and write disjoint data, so
    # updating them from one snapshot equals updating them one after the other.
    p, w = tiny_problem(orc, shape=(14, 8, 9), kz=5, lam=0.02, eta=0.3)
    rz = p.rz
    nsl = [3, 2, 3, 2, 4]
    z0 = np.concatenate([[0], np.cumsum(nsl)[:-1]])
    nc, order, color = orc.color_schedule(nsl, 2 * rz)
    assert nc < len(nsl)
    x = p.y.copy()
    dprev = np.zeros(p.shape)
    p.run(x, dprev, nsl, order, 2, history=False)  # non-trivial state
    for c in range(nc):
        blocks = [b for b in order if color[b] == c]
        xs, ds = x.copy(), dprev.copy()
        for b in blocks:
            p.block_step(xs, ds, int(z0[b]), nsl[b])
        xp, dp = x.copy(), dprev.copy()
        for b in blocks:
            xa, da = x.copy(), dprev.copy()
            p.block_step(xa, da, int(z0[b]), nsl[b])
            sl = slice(int(z0[b]), int(z0[b]) + nsl[b])
            xp[sl], dp[sl] = xa[sl], da[sl]
        assert np.array_equal(xs, xp) and np.array_equal(ds, dp)
        x, dprev = xs, ds
    # and the gap is needed: blocks 1 and 3 are 3 = 2 r_z - 1 slices apart
    assert z0[3] - (z0[1] + nsl[1]) == 2 * rz - 1
    xs, ds = x.copy(), dprev.copy()
    for b in (1, 3):
        p.block_step(xs, ds, int(z0[b]), nsl[b])
    xa, da = x.copy(), dprev.copy()
    p.block_step(xa, da, int(z0[3]), nsl[3])
    sl = slice(int(z0[3]), int(z0[3]) + nsl[3])
    assert not np.array_equal(xa[sl], xs[sl])


def test_orders_reach_same_minimum(orc):
    p, w = tiny_problem(orc, shape=(8, 8, 8), lam=0.02, delta=0.05, eta=0.3)
    nsl = [2, 2, 3, 1]
    nc, corder, _ = orc.color_schedule(nsl, 2 * p.rz)
    res = []
    for order in ([0, 1, 2, 3], corder):
        x = p.y.copy()
        dprev = np.zeros(p.shape)
        s, fh, gh = p.run(x, dprev, nsl, order, 3000, grad_rtol=1e-11)
        res.append((x, fh[-1]))
    assert np.isclose(res[0][1], res[1][1], rtol=1e-12)
    assert np.linalg.norm(res[0][0] - res[1][0]) <= 1e-8 * np.linalg.norm(res[0][0])


def test_resume_is_bitwise(orc):
    p, w = tiny_problem(orc, shape=(8, 8, 8))
    nsl = [2, 2, 4]
    order = [0, 2, 1]
    xa, da = p.y.copy(), np.zeros(p.shape)
    p.run(xa, da, nsl, order, 10, history=False)
    xb, db = p.y.copy(), np.zeros(p.shape)
    p.run(xb, db, nsl, order, 4, history=False)
    p.run(xb, db, nsl, order, 6, history=False)
    assert np.array_equal(xa, xb) and np.array_equal(da, db)


def test_stop_rule_and_history(orc):
    p, w = tiny_problem(orc, shape=(6, 8, 8))
    nsl = [3, 3]
    x, d = p.y.copy(), np.zeros(p.shape)
    g0 = p.grad_norm(p.y)
    s, fh, gh = p.run(x, d, nsl, [0, 1], 500, grad_rtol=2e-3, gnorm_ref=g0)
    assert s < 500 and gh[-1] <= 2e-3 * g0 and np.all(gh[:-1] > 2e-3 * g0)
    assert np.all(np.diff(fh) <= 1e-13 * abs(fh[0]))
    assert np.isclose(fh[-1], p.f(x), rtol=0, atol=0)
