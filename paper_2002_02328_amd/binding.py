"""Thin ctypes binding of libbd3mg (include/bd3mg.h), same function names.

Argument marshalling only: every step of the method runs in the HIP library.
Volumes cross as numpy arrays (host) or as raw device addresses (integers, with
on_device=True), in the problem's storage type (float64 for FP64, float32 for
FP32), shape (nz, ny, nx), C order.  A failing call raises Bd3mgError with the
library's message; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libbd3mg.so")

FP64, FP32 = 0, 1
SCHED_COLORED, SCHED_SEQUENTIAL, SCHED_ROUND = 0, 1, 2
OP_H, OP_HT, OP_GRAD = 0, 1, 2
OK, ERR_ARG, ERR_STATE, ERR_NOMEM, ERR_HIP, ERR_NOT_CONVERGED = range(6)
CHECK_ADAPTIVE = -1  # check_every of run(): checks spaced by the trend of ||grad f||
METHOD_BD3MG, METHOD_ASYNC_GD, METHOD_ASYNC_CG, METHOD_ASYNC_MM = 0, 1, 2, 3
BATCH_AUTO, BATCH_FUSED, BATCH_BRANCHES = 0, 1, 2
OPT_REFRESH_EVERY, OPT_PROFILE = 0, 1
OPT_TILE_ROWS_DIRS, OPT_TILE_ROWS_UPDATE, OPT_TILE_ROWS_AUX, OPT_DIRS_SLICES = 2, 3, 4, 5
OPT_HDP_EVERY = 6
OPT_ROUND_GUARD = 7
OPT_STREAM_STORES = 8
KERNEL_KINDS = ("grad", "dirs", "solve", "update", "eval")

# Every function the header declares, with its C signature.
_dp, _i, _d = C.c_void_p, C.c_int, C.c_double
SIGNATURES = {
    "bd3mg_version": ([], C.c_int),
    "bd3mg_last_error": ([], C.c_char_p),
    "bd3mg_psf_gaussian": ([_i, _i, _dp, _dp], C.c_int),
    "bd3mg_create": ([_i, _i, _i, _i, _dp, C.POINTER(_dp)], C.c_int),
    "bd3mg_destroy": ([_dp], C.c_int),
    "bd3mg_set_psf_separable": ([_dp, _i, _i, _i, _dp, _dp, _dp], C.c_int),
    "bd3mg_set_psf_gaussian": ([_dp, _i, _i, _dp, _dp], C.c_int),
    "bd3mg_psf_rotated_gaussian": ([_i, _i, _i, _dp, _dp, _dp, _dp, _dp], C.c_int),
    "bd3mg_set_psf_dense": ([_dp, _i, _i, _i, _dp], C.c_int),
    "bd3mg_set_params": ([_dp, _d, _d, _d, _d, _d, _d], C.c_int),
    "bd3mg_set_data": ([_dp, _dp, _i], C.c_int),
    "bd3mg_set_blocks": ([_dp, _i, _dp, _i], C.c_int),
    "bd3mg_get_schedule": ([_dp, _dp, _dp, _dp], C.c_int),
    "bd3mg_set_x0": ([_dp, _dp, _i], C.c_int),
    "bd3mg_run": ([_dp, _i, _d, _i, _dp], C.c_int),
    "bd3mg_run_noalloc": ([_dp, _i, _d, _i, _dp], C.c_int),
    "bd3mg_set_method": ([_dp, _i, _d, _i, _d], C.c_int),
    "bd3mg_set_tv3d": ([_dp, _i], C.c_int),
    "bd3mg_round_guard_info": ([_dp, C.POINTER(C.c_int), C.POINTER(C.c_double)], C.c_int),
    "bd3mg_batch_set_mode": ([_dp, _i, _dp], C.c_int),
    "bd3mg_get_x": ([_dp, _dp, _i], C.c_int),
    "bd3mg_get_dprev": ([_dp, _dp, _i], C.c_int),
    "bd3mg_get_state": ([_dp, _dp, _dp, _dp, _dp, _i], C.c_int),
    "bd3mg_set_state": ([_dp, _dp, _dp, _dp, C.c_longlong, _i], C.c_int),
    "bd3mg_set_option": ([_dp, _i, C.c_longlong], C.c_int),
    "bd3mg_get_profile": ([_dp, _dp, _dp, _dp, _i], C.c_int),
    "bd3mg_autotune": ([_dp, _i, _dp, _dp], C.c_int),
    "bd3mg_eval": ([_dp, _dp, _dp], C.c_int),
    "bd3mg_apply": ([_dp, _i, _dp, _dp, _i], C.c_int),
    "bd3mg_block_step": ([_dp, _i, _dp], C.c_int),
    "bd3mg_probe_copy": ([C.c_size_t, _i, _dp, _dp], C.c_int),
    "bd3mg_batch_create": ([_i, _dp, C.POINTER(_dp)], C.c_int),
    "bd3mg_batch_destroy": ([_dp], C.c_int),
    "bd3mg_batch_tune": ([_dp], C.c_int),
    "bd3mg_batch_run": ([_dp, _i, _d, _i, _dp], C.c_int),
    "bd3mg_set_inflation": ([_dp, _d], C.c_int),
    "bd3mg_lipschitz_bound": ([_dp, _dp], C.c_int),
    "bd3mg_net_create": ([_i, _i, _i, C.POINTER(_dp)], C.c_int),
    "bd3mg_net_destroy": ([_dp], C.c_int),
    "bd3mg_net_num_params": ([_dp, C.POINTER(C.c_size_t)], C.c_int),
    "bd3mg_net_set_params": ([_dp, _dp, C.c_size_t], C.c_int),
    "bd3mg_net_get_params": ([_dp, _dp, C.c_size_t], C.c_int),
    "bd3mg_net_save": ([_dp, _dp, C.POINTER(C.c_size_t)], C.c_int),
    "bd3mg_net_load": ([_dp, _dp, C.c_size_t], C.c_int),
    "bd3mg_net_forward": ([_dp, _i, _i, _i, _i, _dp, _dp, _i], C.c_int),
    "bd3mg_net_infer": ([_dp, _dp], C.c_int),
    "bd3mg_net_grad": ([_dp, _i, _i, _i, _i, _dp, _dp, _i, _dp, _dp], C.c_int),
    "bd3mg_net_train_step": ([_dp, _i, _i, _i, _i, _dp, _dp, _i, C.c_float, _dp], C.c_int),
}


class Bd3mgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("bd3mg status %d: %s" % (status, msg))
        self.status = status


class Result(C.Structure):
    _fields_ = [("sweeps", C.c_int), ("converged", C.c_int), ("f", C.c_double),
                ("grad_norm", C.c_double), ("grad_norm_ref", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIBPATH):
    """Load libbd3mg.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError("libbd3mg.so is not built: run __graft_entry__.build() or "
                              "python paper_2002_02328_amd/build.py")
        L = C.CDLL(path)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(status, allow=()):
    if status != OK and status not in allow:
        raise Bd3mgError(status, load().bd3mg_last_error().decode())
    return status


def psf_gaussian(sigma, k):
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    out = np.empty((s.size, k), dtype=np.float64)
    _check(load().bd3mg_psf_gaussian(s.size, k, s.ctypes.data, out.ctypes.data))
    return out


def psf_rotated_gaussian(sx, sy, theta, sz, kxy, kz):
    """[nz][kz][kxy][kxy] per-depth rotated Gaussian kernels (host)."""
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (sx, sy, theta, sz)]
    nz = a[0].size
    if any(v.size != nz for v in a):
        raise ValueError("need one value of each parameter per slice")
    out = np.empty((nz, kz, kxy, kxy), dtype=np.float64)
    _check(load().bd3mg_psf_rotated_gaussian(nz, kxy, kz, *[v.ctypes.data for v in a], out.ctypes.data))
    return out


def probe_copy(nbytes, iters=5):
    """(GB/s, ms) of the best of iters streaming copies of nbytes."""
    gb, ms = C.c_double(), C.c_double()
    _check(load().bd3mg_probe_copy(int(nbytes), int(iters), C.byref(gb), C.byref(ms)))
    return gb.value, ms.value


class Problem:
    """Handle of one BD3MG problem living on the GPU."""

    def __init__(self, nx, ny, nz, precision=FP32, stream=None):
        """stream: None for a stream of the problem's own, or the integer
        handle of a caller's HIP stream (e.g. torch.cuda.Stream().cuda_stream)."""
        L = load()
        h = _dp()
        _check(L.bd3mg_create(nx, ny, nz, precision, None if stream is None else C.c_void_p(int(stream)),
                              C.byref(h)))
        self.stream = stream
        self._h = h
        self.shape = (nz, ny, nx)
        self.precision = precision
        self.dtype = np.float64 if precision == FP64 else np.float32

    def close(self):
        if getattr(self, "_h", None):
            load().bd3mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # marshalling -----------------------------------------------------------
    def _vol_in(self, a, on_device):
        if on_device:
            return C.c_void_p(int(a)), None
        arr = np.ascontiguousarray(a, dtype=self.dtype)
        if arr.shape != self.shape:
            raise ValueError("volume shape %s != %s" % (arr.shape, self.shape))
        return C.c_void_p(arr.ctypes.data), arr

    def _vol_out(self):
        return np.empty(self.shape, dtype=self.dtype)

    # interface ---------------------------------------------------------------
    def set_psf_separable(self, gx, gy, gz):
        gx, gy, gz = (np.ascontiguousarray(t, dtype=np.float64) for t in (gx, gy, gz))
        for t in (gx, gy, gz):
            if t.ndim != 2 or t.shape[0] != self.shape[0]:
                raise ValueError("PSF tables must be [nz][k]")
        _check(load().bd3mg_set_psf_separable(self._h, gx.shape[1], gy.shape[1], gz.shape[1],
                                              gx.ctypes.data, gy.ctypes.data, gz.ctypes.data))

    def set_psf_gaussian(self, kxy, kz, sigma_xy, sigma_z):
        sxy = np.ascontiguousarray(sigma_xy, dtype=np.float64)
        sz = np.ascontiguousarray(sigma_z, dtype=np.float64)
        if sxy.size != self.shape[0] or sz.size != self.shape[0]:
            raise ValueError("need one sigma per slice")
        _check(load().bd3mg_set_psf_gaussian(self._h, kxy, kz, sxy.ctypes.data, sz.ctypes.data))

    def set_psf_dense(self, P):
        """General per-depth kernels P[nz][kz][ky][kx]."""
        P = np.ascontiguousarray(P, dtype=np.float64)
        if P.ndim != 4 or P.shape[0] != self.shape[0]:
            raise ValueError("kernels must be [nz][kz][ky][kx]")
        _check(load().bd3mg_set_psf_dense(self._h, P.shape[3], P.shape[2], P.shape[1], P.ctypes.data))

    def set_params(self, lam, delta, eta, kappa=0.0, xmin=0.0, xmax=1.0):
        _check(load().bd3mg_set_params(self._h, lam, delta, eta, kappa, xmin, xmax))

    def set_method(self, method, lip=0.0, n_inner=1, tol_inner=0.0):
        """Block step of the ablation study: METHOD_BD3MG, METHOD_ASYNC_GD,
        METHOD_ASYNC_CG (metric L Id; lip <= 0: the Lipschitz bound) or
        METHOD_ASYNC_MM (n_inner conjugate-gradient iterations at most)."""
        _check(load().bd3mg_set_method(self._h, int(method), float(lip), int(n_inner), float(tol_inner)))

    def set_tv3d(self, on=True):
        """Total variation over (V^X, V^Y, V^Z) inside the root instead of the
        slices' (V^X, V^Y); kappa ||V^Z x||^2 stays a term of its own."""
        _check(load().bd3mg_set_tv3d(self._h, int(on)))

    def round_guard_info(self):
        """(restores by the last run's guard of the rounds, inflation mu now)."""
        t, mu = C.c_int(), C.c_double()
        _check(load().bd3mg_round_guard_info(self._h, C.byref(t), C.byref(mu)))
        return t.value, mu.value

    def set_inflation(self, mu):
        _check(load().bd3mg_set_inflation(self._h, float(mu)))

    def lipschitz_bound(self):
        L = C.c_double()
        _check(load().bd3mg_lipschitz_bound(self._h, C.byref(L)))
        return L.value

    def set_data(self, y, on_device=False):
        ptr, keep = self._vol_in(y, on_device)
        _check(load().bd3mg_set_data(self._h, ptr, int(on_device)))

    def set_blocks(self, nslices, schedule=SCHED_COLORED):
        ns = np.ascontiguousarray(nslices, dtype=np.int32)
        _check(load().bd3mg_set_blocks(self._h, ns.size, ns.ctypes.data, schedule))
        self.nblocks = ns.size

    def get_schedule(self):
        nc = C.c_int()
        order = np.zeros(self.nblocks, np.int32)
        color = np.zeros(self.nblocks, np.int32)
        _check(load().bd3mg_get_schedule(self._h, C.byref(nc), order.ctypes.data, color.ctypes.data))
        return nc.value, order, color

    def set_x0(self, x0=None, on_device=False):
        if x0 is None:
            _check(load().bd3mg_set_x0(self._h, None, 0))
        else:
            ptr, keep = self._vol_in(x0, on_device)
            _check(load().bd3mg_set_x0(self._h, ptr, int(on_device)))

    def run(self, max_sweeps, grad_rtol=0.0, check_every=None):
        """check_every None: every sweep when grad_rtol > 0, else once at the end."""
        if check_every is None:
            check_every = 1 if grad_rtol > 0 else max(int(max_sweeps), 1)
        res = Result()
        _check(load().bd3mg_run(self._h, max_sweeps, grad_rtol, check_every, C.byref(res)),
               allow=(ERR_NOT_CONVERGED,))
        return res.as_dict()

    def run_noalloc(self, max_sweeps, grad_rtol=0.0, check_every=None):
        """bd3mg_run_noalloc: run with the library's fixed scratch array (no
        device allocation); the schedule must be built (get_schedule)."""
        if check_every is None:
            check_every = 1 if grad_rtol > 0 else max(int(max_sweeps), 1)
        res = Result()
        _check(load().bd3mg_run_noalloc(self._h, max_sweeps, grad_rtol, check_every, C.byref(res)),
               allow=(ERR_NOT_CONVERGED,))
        return res.as_dict()

    def get_x(self, out_ptr=None):
        if out_ptr is not None:
            _check(load().bd3mg_get_x(self._h, C.c_void_p(int(out_ptr)), 1))
            return None
        out = self._vol_out()
        _check(load().bd3mg_get_x(self._h, out.ctypes.data, 0))
        return out

    def get_dprev(self):
        out = self._vol_out()
        _check(load().bd3mg_get_dprev(self._h, out.ctypes.data, 0))
        return out

    def get_state(self):
        """(x, dprev, r, sweeps): everything a bitwise resume needs."""
        x, d, r = self._vol_out(), self._vol_out(), self._vol_out()
        n = C.c_longlong()
        _check(load().bd3mg_get_state(self._h, x.ctypes.data, d.ctypes.data, r.ctypes.data,
                                      C.byref(n), 0))
        return x, d, r, n.value

    def set_state(self, x, dprev, r=None, sweeps=0):
        xp, k1 = self._vol_in(x, False)
        dp, k2 = self._vol_in(dprev, False)
        rp, k3 = self._vol_in(r, False) if r is not None else (None, None)
        _check(load().bd3mg_set_state(self._h, xp, dp, rp, int(sweeps), 0))

    def set_option(self, option, value):
        _check(load().bd3mg_set_option(self._h, option, int(value)))

    def autotune(self, sweeps=5):
        """Pick the fastest tile heights on this problem; returns ((dirs, update), ms/sweep)."""
        ch = np.zeros(2, np.int32)
        ms = C.c_double()
        _check(load().bd3mg_autotune(self._h, int(sweeps), ch.ctypes.data, C.byref(ms)))
        return (int(ch[0]), int(ch[1])), ms.value

    def get_profile(self, reset=False):
        """{kind: (launches, ms, algorithmic bytes)} of the profiled runs."""
        n = np.zeros(len(KERNEL_KINDS), np.int64)
        ms = np.zeros(len(KERNEL_KINDS))
        by = np.zeros(len(KERNEL_KINDS))
        _check(load().bd3mg_get_profile(self._h, n.ctypes.data, ms.ctypes.data, by.ctypes.data,
                                        int(reset)))
        return {k: (int(n[i]), float(ms[i]), float(by[i])) for i, k in enumerate(KERNEL_KINDS)}

    def eval(self):
        f, g = C.c_double(), C.c_double()
        _check(load().bd3mg_eval(self._h, C.byref(f), C.byref(g)))
        return f.value, g.value

    def apply(self, op, v):
        ptr, keep = self._vol_in(v, False)
        out = self._vol_out()
        _check(load().bd3mg_apply(self._h, op, ptr, out.ctypes.data, 0))
        return out

    def H(self, v):
        return self.apply(OP_H, v)

    def HT(self, v):
        return self.apply(OP_HT, v)

    def grad(self, v):
        return self.apply(OP_GRAD, v)

    def block_step(self, b):
        info = np.zeros(8)
        _check(load().bd3mg_block_step(self._h, b, info.ctypes.data))
        return info


class Batch:
    """Several fully set-up problems advanced together (one HIP graph launch
    runs two sweeps of every problem).  Keeps references to its problems."""

    def __init__(self, problems):
        self.problems = list(problems)
        arr = (_dp * len(self.problems))(*[p._h for p in self.problems])
        h = _dp()
        _check(load().bd3mg_batch_create(len(self.problems), arr, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().bd3mg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tune(self):
        _check(load().bd3mg_batch_tune(self._h))

    def set_mode(self, mode):
        """BATCH_AUTO, BATCH_FUSED or BATCH_BRANCHES; returns whether fused
        launches will run."""
        f = C.c_int()
        _check(load().bd3mg_batch_set_mode(self._h, int(mode), C.byref(f)))
        return bool(f.value)

    def run(self, max_sweeps, grad_rtol=0.0, check_every=0):
        res = (Result * len(self.problems))()
        _check(load().bd3mg_batch_run(self._h, int(max_sweeps), float(grad_rtol), int(check_every), res),
               allow=(ERR_NOT_CONVERGED,))
        return [r.as_dict() for r in res]


class Net:
    """Handle of the warm-start network x0 = y + net(y) (three-level 3D U-Net,
    16 base channels, bf16 matrix-core kernels).  Volumes are float32 arrays
    (nb, nz, ny, nx) or (nz, ny, nx) on the host, or device addresses with
    on_device=True and an explicit shape."""

    def __init__(self, levels=3, base_channels=16, in_channels=1):
        h = _dp()
        _check(load().bd3mg_net_create(levels, base_channels, in_channels, C.byref(h)))
        self._h = h
        n = C.c_size_t()
        _check(load().bd3mg_net_num_params(self._h, C.byref(n)))
        self.num_params = n.value

    def close(self):
        if getattr(self, "_h", None):
            load().bd3mg_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32).ravel()
        _check(load().bd3mg_net_set_params(self._h, p.ctypes.data, p.size))

    def get_params(self):
        p = np.empty(self.num_params, dtype=np.float32)
        _check(load().bd3mg_net_get_params(self._h, p.ctypes.data, p.size))
        return p

    def save(self):
        n = C.c_size_t()
        _check(load().bd3mg_net_save(self._h, None, C.byref(n)))
        buf = (C.c_char * n.value)()
        _check(load().bd3mg_net_save(self._h, buf, C.byref(n)))
        return bytes(buf[:n.value])

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(load().bd3mg_net_load(self._h, buf, len(blob)))

    @staticmethod
    def _batch(a, shape, on_device):
        if on_device:
            nb, nz, ny, nx = shape
            return C.c_void_p(int(a)), None, (nb, nz, ny, nx)
        arr = np.ascontiguousarray(a, dtype=np.float32)
        if arr.ndim == 3:
            arr = arr[None]
        if arr.ndim != 4:
            raise ValueError("expected (nb, nz, ny, nx) or (nz, ny, nx)")
        return C.c_void_p(arr.ctypes.data), arr, arr.shape

    def forward(self, y, on_device=False, shape=None, out=None):
        ptr, keep, (nb, nz, ny, nx) = self._batch(y, shape, on_device)
        if on_device:
            _check(load().bd3mg_net_forward(self._h, nb, nx, ny, nz, ptr, C.c_void_p(int(out)), 1))
            return out
        res = np.empty((nb, nz, ny, nx), dtype=np.float32)
        _check(load().bd3mg_net_forward(self._h, nb, nx, ny, nz, ptr, res.ctypes.data, 0))
        return res if np.ndim(y) == 4 else res[0]

    def infer(self, problem):
        """Set problem's start point to y + net(y)."""
        _check(load().bd3mg_net_infer(self._h, problem._h))

    def grad(self, y, xstar, on_device=False, shape=None):
        py, ky, sh = self._batch(y, shape, on_device)
        pt, kt, sh2 = self._batch(xstar, shape, on_device)
        if sh != sh2:
            raise ValueError("y and xstar shapes differ")
        nb, nz, ny, nx = sh
        g = np.empty(self.num_params, dtype=np.float32)
        loss = C.c_double()
        _check(load().bd3mg_net_grad(self._h, nb, nx, ny, nz, py, pt, int(on_device), g.ctypes.data,
                                     C.byref(loss)))
        return loss.value, g

    def train_step(self, y, xstar, lr, on_device=False, shape=None, want_loss=True):
        py, ky, sh = self._batch(y, shape, on_device)
        pt, kt, sh2 = self._batch(xstar, shape, on_device)
        if sh != sh2:
            raise ValueError("y and xstar shapes differ")
        nb, nz, ny, nx = sh
        loss = C.c_double()
        _check(load().bd3mg_net_train_step(self._h, nb, nx, ny, nz, py, pt, int(on_device), float(lr),
                                           C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None
