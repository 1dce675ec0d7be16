"""FP64 CPU oracle for BD3MG (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The product library never does, and the two share no
code.  Every function here wraps the plain C implementation in
``bd3mg_oracle.c`` (built by ``oracle/build.py``) and takes float64 numpy
volumes laid out [nz][ny][nx], x fastest.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB lets the mutation test load a deliberately broken build.
LIBPATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

_lib = None


class _Problem(C.Structure):
    _fields_ = [
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("kx", C.c_int), ("ky", C.c_int), ("kz", C.c_int),
        ("gx", C.c_void_p), ("gy", C.c_void_p), ("gz", C.c_void_p),
        ("y", C.c_void_p),
        ("lam", C.c_double), ("delta", C.c_double), ("eta", C.c_double),
        ("kappa", C.c_double), ("xmin", C.c_double), ("xmax", C.c_double),
        ("dense", C.c_int),
        ("mu", C.c_double),
        ("pk", C.c_void_p),
        ("method", C.c_int),
        ("lip", C.c_double),
        ("n_inner", C.c_int),
        ("tol_inner", C.c_double),
        ("tv3d", C.c_int),
    ]

# Block steps of the ablation study (Sec. 3.2): BD3MG and its variants.
BD3MG, ASYNC_GD, ASYNC_CG, ASYNC_MM = 0, 1, 2, 3


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIBPATH)
        P = C.POINTER(_Problem)
        dp = C.c_void_p
        L.orc_gauss_table.argtypes = [C.c_int, C.c_int, dp, dp]
        L.orc_rotated_gauss.argtypes = [C.c_int, C.c_int, C.c_int, dp, dp, dp, dp, dp]
        L.orc_H.argtypes = [P, dp, dp, C.c_int, C.c_int]
        L.orc_HT.argtypes = [P, dp, dp, C.c_int, C.c_int]
        L.orc_V.argtypes = [P, C.c_int, C.c_int, dp, dp]
        L.orc_f_terms.argtypes = [P, dp, dp]
        L.orc_f_terms.restype = C.c_double
        L.orc_f.argtypes = [P, dp]
        L.orc_f.restype = C.c_double
        L.orc_grad_slices.argtypes = [P, dp, dp, C.c_int, C.c_int]
        L.orc_grad.argtypes = [P, dp, dp]
        L.orc_grad_norm.argtypes = [P, dp]
        L.orc_grad_norm.restype = C.c_double
        L.orc_dot.argtypes = [P, dp, dp]
        L.orc_dot.restype = C.c_double
        L.orc_majorant_form.argtypes = [P, dp, dp, dp, C.c_int, C.c_int]
        L.orc_majorant_form.restype = C.c_double
        L.orc_majorant_apply.argtypes = [P, dp, dp, dp, C.c_int, C.c_int]
        L.orc_pinv2.argtypes = [dp, dp]
        L.orc_color_schedule.argtypes = [C.c_int, dp, C.c_int, dp, dp]
        L.orc_color_schedule.restype = C.c_int
        L.orc_block_step.argtypes = [P, dp, dp, C.c_int, C.c_int, dp]
        L.orc_run.argtypes = [P, dp, dp, C.c_int, dp, dp, C.c_int, C.c_double, C.c_double, dp, dp]
        L.orc_run.restype = C.c_int
        L.orc_run_round.argtypes = [P, dp, dp, C.c_int, dp, C.c_int, C.c_double, C.c_double, dp, dp]
        L.orc_run_round.restype = C.c_int
        L.orc_lipschitz_bound.argtypes = [P]
        L.orc_lipschitz_bound.restype = C.c_double
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        L.orcnet_num_params.argtypes = [C.c_int, C.c_int]
        L.orcnet_num_params.restype = C.c_size_t
        L.orcnet_round_bf16.argtypes = [C.c_double]
        L.orcnet_round_bf16.restype = C.c_double
        L.orcnet_forward.argtypes = [C.c_int, C.c_int, dp, dp, C.c_int, C.c_int, C.c_int, C.c_int, dp]
        L.orcnet_loss_grad.argtypes = [C.c_int, C.c_int, dp, dp, dp, C.c_int, C.c_int, C.c_int, C.c_int, dp]
        L.orcnet_loss_grad.restype = C.c_double
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of later oracle calls (OpenMP)."""
    lib().orc_set_num_threads(int(n))


def gauss_table(sigma, k: int) -> np.ndarray:
    """[nz][k] normalised 1-D Gaussian factors for per-slice sigma (Sec. 3.1)."""
    s = _f64(sigma)
    out = np.empty((s.size, k), dtype=np.float64)
    lib().orc_gauss_table(int(s.size), int(k), _ptr(s), _ptr(out))
    return out


def rotated_gauss_kernels(sx, sy, theta, sz, kxy: int, kz: int) -> np.ndarray:
    """[nz][kz][kxy][kxy] per-depth rotated anisotropic Gaussians, each summing
    to 1 (the blur of the paper's experiments, Sec. 3.1: variance and rotation
    drawn per depth)."""
    a = [_f64(v) for v in (sx, sy, theta, sz)]
    nz = a[0].size
    assert all(v.size == nz for v in a)
    out = np.empty((nz, kz, kxy, kxy), dtype=np.float64)
    lib().orc_rotated_gauss(int(nz), int(kxy), int(kz), *[_ptr(v) for v in a], _ptr(out))
    return out


class Problem:
    """The criterion of Sec. 3.1 on one volume, with a depth-variant PSF.

    gx, gy, gz: [nz][K] factor tables of a separable PSF; y: [nz][ny][nx]
    observation.  dense=True evaluates H by its triple-sum definition,
    otherwise by the separable twin.  Problem.with_kernels takes general
    per-slice kernels instead.
    """

    @classmethod
    def with_kernels(cls, y, pk, **kw):
        """General per-slice kernels pk[nz][kz][ky][kx] (odd sizes), applied
        by the triple sum (Hx)_k = sum_{c,b,a} pk[k][c][b][a] x_{k-c,j-b,i-a}."""
        pk = _f64(pk)
        nz = np.asarray(y).shape[0]
        assert pk.ndim == 4 and pk.shape[0] == nz and all(n % 2 == 1 for n in pk.shape[1:])
        kz, ky, kx = pk.shape[1:]
        o = cls(y, np.zeros((nz, kx)), np.zeros((nz, ky)), np.zeros((nz, kz)), **kw)
        o.pk = pk
        o._s.pk = pk.ctypes.data
        return o

    def __init__(self, y, gx, gy, gz, lam=0.0, delta=1.0, eta=0.0, kappa=0.0,
                 xmin=0.0, xmax=1.0, dense=False, mu=0.0, tv3d=False):
        """method etc.: see set_method (BD3MG unless changed).  tv3d: V^Z inside
        the root of the TV term with V^X and V^Y."""
        self.y = _f64(y)
        assert self.y.ndim == 3
        self.nz, self.ny, self.nx = self.y.shape
        self.gx, self.gy, self.gz = _f64(gx), _f64(gy), _f64(gz)
        for g in (self.gx, self.gy, self.gz):
            assert g.ndim == 2 and g.shape[0] == self.nz and g.shape[1] % 2 == 1
        self.lam, self.delta, self.eta, self.kappa = float(lam), float(delta), float(eta), float(kappa)
        self.xmin, self.xmax = float(xmin), float(xmax)
        self.dense = bool(dense)
        self.mu = float(mu)
        self._s = _Problem(self.nx, self.ny, self.nz,
                           self.gx.shape[1], self.gy.shape[1], self.gz.shape[1],
                           self.gx.ctypes.data, self.gy.ctypes.data, self.gz.ctypes.data,
                           self.y.ctypes.data, self.lam, self.delta, self.eta, self.kappa,
                           self.xmin, self.xmax, int(self.dense), self.mu, None,
                           BD3MG, 0.0, 0, 0.0, int(bool(tv3d)))
        self.tv3d = bool(tv3d)
        self.pk = None

    def set_method(self, method, lip=None, n_inner=10, tol_inner=0.0):
        """Block step of the ablation study (Sec. 3.2): BD3MG, ASYNC_GD (step
        -grad / L), ASYNC_CG (BD3MG's subspace [-grad, d_prev] with the metric
        L Id, which gives Async-GD's step up to rounding) or
        ASYNC_MM (d' = -A_S(x)^{-1} grad_S f by at most n_inner BiCG
        iterations, stopping once ||r|| <= tol_inner ||r_0||).  lip: L of the
        metric L Id (default: the Lipschitz bound of grad f)."""
        self._s.method = int(method)
        self._s.lip = float(self.lipschitz_bound() if lip is None else lip)
        self._s.n_inner = int(n_inner)
        self._s.tol_inner = float(tol_inner)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def rz(self):
        return self.gz.shape[1] // 2

    def _p(self):
        return C.byref(self._s)

    def H(self, x, k0=0, k1=None):
        x = _f64(x)
        out = np.zeros(self.shape)
        lib().orc_H(self._p(), _ptr(x), _ptr(out), int(k0), int(self.nz if k1 is None else k1))
        return out

    def HT(self, r, k0=0, k1=None):
        r = _f64(r)
        out = np.zeros(self.shape)
        lib().orc_HT(self._p(), _ptr(r), _ptr(out), int(k0), int(self.nz if k1 is None else k1))
        return out

    def V(self, x, axis: str, adjoint=False):
        x = _f64(x)
        out = np.empty(self.shape)
        lib().orc_V(self._p(), {"x": 0, "y": 1, "z": 2}[axis], int(adjoint), _ptr(x), _ptr(out))
        return out

    def f(self, x):
        x = _f64(x)
        return float(lib().orc_f(self._p(), _ptr(x)))

    def f_terms(self, x):
        x = _f64(x)
        t = np.zeros(4)
        lib().orc_f_terms(self._p(), _ptr(x), _ptr(t))
        return t

    def grad(self, x, k0=None, k1=None):
        x = _f64(x)
        g = np.zeros(self.shape)
        if k0 is None:
            lib().orc_grad(self._p(), _ptr(x), _ptr(g))
        else:
            lib().orc_grad_slices(self._p(), _ptr(x), _ptr(g), int(k0), int(k1))
        return g

    def grad_norm(self, x):
        x = _f64(x)
        return float(lib().orc_grad_norm(self._p(), _ptr(x)))

    def majorant_form(self, x, u, v, z0=0, z1=None):
        x, u, v = _f64(x), _f64(u), _f64(v)
        return float(lib().orc_majorant_form(self._p(), _ptr(x), _ptr(u), _ptr(v),
                                             int(z0), int(self.nz if z1 is None else z1)))

    def majorant_apply(self, x, u, z0=0, z1=None):
        """[A(x) u]_S for u supported on the slices [z0, z1) (zero elsewhere;
        plus mu u): the principal submatrix of the majorant times u."""
        x, u = _f64(x), _f64(u)
        out = np.zeros(self.shape)
        lib().orc_majorant_apply(self._p(), _ptr(x), _ptr(u), _ptr(out), int(z0),
                                 int(self.nz if z1 is None else z1))
        return out

    def block_step(self, x, dprev, z0, n):
        """One worker step plus master update, in place on x and dprev.

        Returns {B11, B12, B22, c1, c2, u1, u2, |g|^2} of the step."""
        assert x.dtype == np.float64 and x.flags.c_contiguous
        assert dprev.dtype == np.float64 and dprev.flags.c_contiguous
        info = np.zeros(8)
        lib().orc_block_step(self._p(), _ptr(x), _ptr(dprev), int(z0), int(n), _ptr(info))
        return info

    def run(self, x, dprev, nslices, order, max_sweeps, grad_rtol=0.0, gnorm_ref=None,
            history=True):
        """BD3MG sweeps in the given block order; x, dprev updated in place.

        Returns (sweeps, f_hist, g_hist)."""
        assert x.dtype == np.float64 and x.flags.c_contiguous
        assert dprev.dtype == np.float64 and dprev.flags.c_contiguous
        ns = np.ascontiguousarray(nslices, dtype=np.int32)
        od = np.ascontiguousarray(order, dtype=np.int32)
        assert ns.sum() == self.nz
        if gnorm_ref is None:
            gnorm_ref = self.grad_norm(self.y) if grad_rtol > 0 else 0.0
        fh = np.full(max_sweeps, np.nan) if history else None
        gh = np.full(max_sweeps, np.nan) if history else None
        s = lib().orc_run(self._p(), _ptr(x), _ptr(dprev), int(ns.size), _ptr(ns), _ptr(od),
                          int(max_sweeps), float(grad_rtol), float(gnorm_ref),
                          _ptr(fh) if history else None, _ptr(gh) if history else None)
        if history:
            return s, fh[:s], gh[:s]
        return s, None, None

    def run_round(self, x, dprev, nslices, max_sweeps, grad_rtol=0.0, gnorm_ref=None,
                  history=True):
        """Asynchronous rounds: every block steps from the same snapshot (each
        majorant inflated by the problem's mu Id); x, dprev updated in place.

        Returns (sweeps, f_hist, g_hist)."""
        assert x.dtype == np.float64 and x.flags.c_contiguous
        assert dprev.dtype == np.float64 and dprev.flags.c_contiguous
        ns = np.ascontiguousarray(nslices, dtype=np.int32)
        assert ns.sum() == self.nz
        if gnorm_ref is None:
            gnorm_ref = self.grad_norm(self.y) if grad_rtol > 0 else 0.0
        fh = np.full(max_sweeps, np.nan) if history else None
        gh = np.full(max_sweeps, np.nan) if history else None
        s = lib().orc_run_round(self._p(), _ptr(x), _ptr(dprev), int(ns.size), _ptr(ns),
                                int(max_sweeps), float(grad_rtol), float(gnorm_ref),
                                _ptr(fh) if history else None, _ptr(gh) if history else None)
        if history:
            return s, fh[:s], gh[:s]
        return s, None, None

    def lipschitz_bound(self):
        """Upper bound of the Lipschitz constant of grad f from the tables."""
        return float(lib().orc_lipschitz_bound(self._p()))


def pinv2(b11, b12, b22):
    B = np.array([b11, b12, b22], dtype=np.float64)
    P = np.zeros(3)
    lib().orc_pinv2(_ptr(B), _ptr(P))
    return np.array([[P[0], P[1]], [P[1], P[2]]])


def color_schedule(nslices, min_gap):
    """(ncolors, order, color) of the coloured sweep for z-slab blocks."""
    ns = np.ascontiguousarray(nslices, dtype=np.int32)
    order = np.zeros(ns.size, dtype=np.int32)
    color = np.zeros(ns.size, dtype=np.int32)
    nc = lib().orc_color_schedule(int(ns.size), _ptr(ns), int(min_gap), _ptr(order), _ptr(color))
    return int(nc), order, color


# ---------------------------------------------------------------------------
# Learned warm start: the three-level 3D U-Net of convnet_oracle.c.
# Volumes are [C][D][H][W] (a [D][H][W] array is one channel); parameters are
# one flat float64 array, layer by layer: weights [Cout][Cin][kd][kh][kw], then
# bias [Cout].  bf16=True rounds stored activations and weights to bfloat16.

NET_LAYERS = 11


def net_layer_shapes(c: int, cin: int = 1):
    """(cout, cin, k) of every layer, in parameter order."""
    return [(c, cin, 3), (c, c, 3), (2 * c, c, 3), (2 * c, 2 * c, 3), (4 * c, 2 * c, 3),
            (4 * c, 4 * c, 3), (2 * c, 4 * c, 3), (2 * c, 4 * c, 3), (c, 2 * c, 3), (c, 2 * c, 3),
            (1, c, 1)]


def net_num_params(c: int, cin: int = 1) -> int:
    return int(lib().orcnet_num_params(c, cin))


def round_bf16(v: float) -> float:
    return float(lib().orcnet_round_bf16(float(v)))


def _vol(x, cin):
    x = _f64(x)
    if x.ndim == 3:
        x = x[None]
    assert x.ndim == 4 and x.shape[0] == cin, x.shape
    assert all(s % 4 == 0 for s in x.shape[1:]), "volume sides must be multiples of 4"
    return np.ascontiguousarray(x)


def net_forward(params, x, c: int, cin: int = 1, bf16: bool = False) -> np.ndarray:
    """x0 = x[channel 0] + net(x); returns [D][H][W]."""
    params = _f64(params)
    assert params.size == net_num_params(c, cin)
    x = _vol(x, cin)
    _, D, H, W = x.shape
    out = np.empty((D, H, W))
    lib().orcnet_forward(c, cin, _ptr(params), _ptr(x), D, H, W, int(bf16), _ptr(out))
    return out


def net_loss_grad(params, x, target, c: int, cin: int = 1, bf16: bool = False):
    """Mean squared error of x[0] + net(x) against target, and its gradient
    with respect to the flat parameters."""
    params = _f64(params)
    assert params.size == net_num_params(c, cin)
    x = _vol(x, cin)
    _, D, H, W = x.shape
    t = _f64(target).reshape(D, H, W)
    g = np.empty(params.size)
    loss = lib().orcnet_loss_grad(c, cin, _ptr(params), _ptr(x), _ptr(t), D, H, W, int(bf16), _ptr(g))
    return float(loss), g
