"""Pins of the oracle's ablation variants (Sec. 3.2, "Ablation study and
comparative analysis", and its table of methods): Async-GD, Async-CG and
Async-MM, each a change of the Worker's step of BD3MG.

Pinned against mathematics and library routines, not against the oracle's
own formulas:
* the majorant matrix applied to a block vector agrees with the bilinear
  form (a separate code path: <Hu, Hv> against H^T H u), is symmetric, and
  its dense assembly from unit vectors equals the form's;
* Async-GD's step is -grad_S f / L exactly;
* Async-CG as the paper defines it (BD3MG's subspace [-g, d_prev] with the
  metric L Id) collapses to that same step -- the minimiser of an isotropic
  model over any subspace holding g is -g / L (numpy's pseudo-inverse) -- and
  the oracle's Async-CG trajectory is Async-GD's up to rounding;
* Async-MM's BiCG solve equals numpy.linalg.solve on the dense block
  majorant, and with lambda = eta = 0 and one block it is a Newton step that
  lands on the normal-equations solution in one sweep;
* with L at least the Lipschitz constant every variant decreases f at every
  block update and all reach the minimiser BD3MG reaches.
"""
import numpy as np
import pytest

from paper_2002_02328_amd import inputs


def tiny(orc, shape=(6, 7, 9), seed=3, lam=0.02, delta=0.05, eta=0.3, kappa=0.0, kxy=3, kz=3, mu=0.0):
    w = inputs.tiny(shape, seed, kxy=kxy, kz=kz, lam=lam, delta=delta, eta=eta, kappa=kappa)
    gx = orc.gauss_table(w.sigma_xy, kxy)
    gz = orc.gauss_table(w.sigma_z, kz)
    y = orc.Problem(np.zeros(shape), gx, gx, gz).H(w.xbar) + w.noise
    return orc.Problem(y, gx, gx, gz, lam=lam, delta=delta, eta=eta, kappa=kappa, mu=mu)


def on_block(v, z0, z1):
    out = np.zeros_like(v)
    out[z0:z1] = v[z0:z1]
    return out


@pytest.mark.parametrize("kappa,mu", [(0.0, 0.0), (0.07, 0.0), (0.05, 0.4)])
def test_majorant_apply_agrees_with_the_form(orc, kappa, mu):
    p = tiny(orc, shape=(7, 8, 10), kappa=kappa, mu=mu, kz=5)
    rng = np.random.default_rng(1)
    x = rng.uniform(-0.2, 1.2, size=p.shape)
    for z0, z1 in [(0, 2), (2, 5), (4, 7), (0, 7)]:
        u = on_block(rng.standard_normal(p.shape), z0, z1)
        v = on_block(rng.standard_normal(p.shape), z0, z1)
        au = p.majorant_apply(x, u, z0, z1)
        av = p.majorant_apply(x, v, z0, z1)
        assert np.all(au[:z0] == 0) and np.all(au[z1:] == 0)
        form = p.majorant_form(x, u, v, z0, z1) + mu * float((u * v).sum())
        assert abs(float((v * au).sum()) - form) <= 1e-12 * abs(form)
        assert abs(float((v * au).sum()) - float((u * av).sum())) <= 1e-12 * abs(form)


def test_majorant_apply_dense_assembly_equals_the_form(orc):
    p = tiny(orc, shape=(3, 4, 5), kappa=0.05)
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, size=p.shape)
    z0, z1 = 1, 3
    idx = [q for q in range(x.size) if z0 <= np.unravel_index(q, p.shape)[0] < z1]
    n = len(idx)
    E = np.zeros((n,) + p.shape)
    for a, q in enumerate(idx):
        E[a].flat[q] = 1.0
    A_form = np.array([[p.majorant_form(x, E[a], E[b], z0, z1) for b in range(n)] for a in range(n)])
    A_apply = np.array([p.majorant_apply(x, E[a], z0, z1).ravel()[idx] for a in range(n)])
    assert np.allclose(A_apply, A_form, rtol=1e-12, atol=1e-14)
    assert np.all(np.linalg.eigvalsh(A_form) > 0)  # positive definite (delta > 0, eta > 0)


def test_async_gd_step_is_the_scaled_gradient(orc):
    p = tiny(orc)
    L = p.lipschitz_bound()
    p.set_method(orc.ASYNC_GD)
    x = p.y.copy()
    d = np.zeros(p.shape)
    for (z0, n) in [(0, 2), (2, 3), (5, 1), (0, 2)]:
        g = p.grad(x)
        x_ref = x - on_block(g, z0, z0 + n) / L
        info = p.block_step(x, d, z0, n)
        assert np.allclose(x, x_ref, rtol=1e-14, atol=1e-16)
        assert abs(info[5] - 1.0 / L) <= 1e-15 / L and info[6] == 0.0


def test_literal_async_cg_collapses_to_async_gd(orc):
    """BD3MG's step u = -(D^T A D)^+ D^T g with A = L Id and D = [-g, d]
    gives D u = -g / L whatever d is (g lies in the range of D)."""
    p = tiny(orc)
    L = p.lipschitz_bound()
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 1, size=p.shape)
    g = on_block(p.grad(x), 1, 4).ravel()
    for d in (rng.standard_normal(g.size), g + 1e-3 * rng.standard_normal(g.size)):
        d = on_block(d.reshape(p.shape), 1, 4).ravel()
        D = np.stack([-g, d], axis=1)
        u = -np.linalg.pinv(L * D.T @ D) @ (D.T @ g)
        assert np.allclose(D @ u, -g / L, rtol=1e-9, atol=1e-12 * np.abs(g).max() / L)


def test_async_cg_trajectory_is_async_gd_up_to_rounding(orc):
    """The oracle's Async-CG (the Worker's 2x2 subspace system with the
    metric L Id) follows Async-GD's trajectory: its memory coefficient is
    rounding, every step decreases f (L at least the Lipschitz constant)."""
    p = tiny(orc, shape=(8, 9, 10))
    pg = tiny(orc, shape=(8, 9, 10))
    p.set_method(orc.ASYNC_CG)
    pg.set_method(orc.ASYNC_GD)
    x, d = p.y.copy(), np.zeros(p.shape)
    xg, dg = p.y.copy(), np.zeros(p.shape)
    nsl = [3, 2, 3]
    z0 = [0, 3, 5]
    for sweep in range(12):
        for b in range(3):
            f0 = p.f(x)
            info = p.block_step(x, d, z0[b], nsl[b])
            pg.block_step(xg, dg, z0[b], nsl[b])
            assert p.f(x) <= f0 + 1e-13 * abs(f0)
            assert abs(info[6]) <= 1e-12 * abs(info[5])
    assert np.linalg.norm(x - xg) <= 1e-13 * np.linalg.norm(xg)


def dense_matrix(op, shape):
    n = int(np.prod(shape))
    M = np.zeros((n, n))
    for q in range(n):
        e = np.zeros(n)
        e[q] = 1.0
        M[:, q] = op(e.reshape(shape)).ravel()
    return M


def test_async_mm_bicg_solves_the_block_system(orc):
    p = tiny(orc, shape=(4, 5, 6), kappa=0.03)
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 1, size=p.shape)
    z0, n = 1, 2
    idx = np.flatnonzero(on_block(np.ones(p.shape), z0, z0 + n).ravel())
    A = np.zeros((idx.size, idx.size))
    for a, q in enumerate(idx):
        e = np.zeros(x.size)
        e[q] = 1.0
        A[:, a] = p.majorant_apply(x, e.reshape(p.shape), z0, z0 + n).ravel()[idx]
    g = p.grad(x).ravel()[idx]
    v = np.linalg.solve(A, -g)
    p.set_method(orc.ASYNC_MM, n_inner=4 * idx.size)
    d = np.zeros(p.shape)
    xs = x.copy()
    p.block_step(xs, d, z0, n)
    assert np.linalg.norm(d.ravel()[idx] - v) <= 1e-9 * np.linalg.norm(v)
    assert np.array_equal(xs - d, x) or np.allclose(xs, x + d, rtol=0, atol=1e-15)
    # few iterations: the truncated solve still decreases f (MM step on a
    # Krylov subspace of the majorant)
    p.set_method(orc.ASYNC_MM, n_inner=2)
    f0 = p.f(x)
    xt, dt = x.copy(), np.zeros(p.shape)
    info = p.block_step(xt, dt, z0, n)
    assert info[0] == 2 and p.f(xt) < f0


def test_async_mm_is_newton_at_zero_regularisation(orc):
    rng = np.random.default_rng(6)
    shape = (4, 4, 5)
    tabs = (orc.gauss_table(np.full(4, 0.5), 3), orc.gauss_table(np.full(4, 0.6), 3),
            orc.gauss_table(np.full(4, 0.7), 3))
    y = rng.uniform(size=shape)
    p = orc.Problem(y, *tabs, lam=0.0, delta=1.0, eta=0.0)
    M = dense_matrix(p.H, shape)
    xs = np.linalg.solve(M.T @ M, M.T @ y.ravel())
    p.set_method(orc.ASYNC_MM, n_inner=400, tol_inner=1e-14)
    x, d = y.copy(), np.zeros(shape)
    p.run(x, d, [4], [0], 1, history=False)
    assert np.linalg.norm(x.ravel() - xs) <= 1e-9 * np.linalg.norm(xs)


@pytest.mark.parametrize("method,sweeps", [("ASYNC_GD", 6000), ("ASYNC_CG", 6000), ("ASYNC_MM", 1000)])
def test_variants_reach_the_bd3mg_minimiser(orc, method, sweeps):
    p = tiny(orc, shape=(6, 8, 8), lam=0.02, delta=0.1, eta=0.3)
    nsl = [2, 3, 1]
    x_ref, d = p.y.copy(), np.zeros(p.shape)
    p.run(x_ref, d, nsl, [0, 1, 2], 20000, grad_rtol=1e-11, history=False)
    assert p.grad_norm(x_ref) <= 1e-11 * p.grad_norm(p.y)
    q = tiny(orc, shape=(6, 8, 8), lam=0.02, delta=0.1, eta=0.3)
    q.set_method(getattr(orc, method), n_inner=20, tol_inner=1e-6)
    x, d = q.y.copy(), np.zeros(q.shape)
    s, fh, gh = q.run(x, d, nsl, [0, 1, 2], sweeps, grad_rtol=1e-7)
    assert np.all(np.diff(fh) <= 1e-13 * np.abs(fh[1:]))  # monotone
    assert np.linalg.norm(x - x_ref) <= 1e-5 * np.linalg.norm(x_ref), (method, s)


def test_round_variants_match_sequential_when_blocks_do_not_interact(orc):
    """kz = 1 and lambda acting in-slice only: blocks do not interact, so a
    round (every block from one snapshot) equals a sequential sweep, for
    every variant (the per-block memory of Async-CG included)."""
    for m in ("ASYNC_GD", "ASYNC_CG", "ASYNC_MM"):
        a = tiny(orc, shape=(5, 6, 7), kz=1)
        b = tiny(orc, shape=(5, 6, 7), kz=1)
        a.set_method(getattr(orc, m), n_inner=5)
        b.set_method(getattr(orc, m), n_inner=5)
        xa, da = a.y.copy(), np.zeros(a.shape)
        xb, db = b.y.copy(), np.zeros(b.shape)
        a.run(xa, da, [2, 1, 2], [0, 1, 2], 4, history=False)
        b.run_round(xb, db, [2, 1, 2], 4, history=False)
        assert np.allclose(xa, xb, rtol=1e-13, atol=1e-15), m
