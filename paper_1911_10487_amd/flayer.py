"""Python binding of the flayer C ABI (include/flayer.h).

Argument marshalling only: device arrays are PyTorch tensors on the GPU
(torch is used for device memory and the current HIP stream); every step of
the inversion runs in the library's HIP kernels. There is no CPU fallback:
if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libflayer.so")

FL_OK, FL_EINVAL, FL_ENOMEM, FL_EDEVICE, FL_ENOCONV, FL_ENUMERIC, FL_EUNSUPPORTED = range(7)
STATUS_NAMES = {0: "FL_OK", 1: "FL_EINVAL", 2: "FL_ENOMEM", 3: "FL_EDEVICE", 4: "FL_ENOCONV",
                5: "FL_ENUMERIC", 6: "FL_EUNSUPPORTED"}
TAP_WHAT, TAP_VHAT, TAP_V, TAP_U, TAP_ALPHA, TAP_BRANCH, TAP_GTAB, TAP_KTAB = range(1, 9)
STAGES = ["norm", "fft_rows", "fft_cols", "classify", "bidiag", "dp", "backtransform",
          "ifft_cols", "crop_pad", "conv_cols", "conv_z", "conv_icols", "conv_irows", "xi"]


class FlError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class FlOpts(ctypes.Structure):
    _fields_ = [
        ("px", ctypes.c_int), ("py", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("tau", ctypes.c_double), ("eta", ctypes.c_double),
        ("combine", ctypes.c_int), ("input_dtype", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("max_chunk", ctypes.c_int),
        ("kernel_mode", ctypes.c_int), ("damping", ctypes.c_double),
        ("alpha_rule", ctypes.c_int), ("factor_per_system", ctypes.c_int),
        ("forward_method", ctypes.c_int), ("prefactor", ctypes.c_int),
        ("regularizer", ctypes.c_int),
        ("hz", ctypes.c_double),
    ]


class FlTuning(ctypes.Structure):
    _fields_ = [("bidiag_variant", ctypes.c_int), ("bidiag_grid", ctypes.c_int),
                ("dp_grid", ctypes.c_int), ("dp_systems_per_wave", ctypes.c_int)]


class FlPlanInfo(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("nd", ctypes.c_int),
        ("px", ctypes.c_int), ("py", ctypes.c_int), ("n_omega", ctypes.c_int),
        ("precision", ctypes.c_int), ("device_bytes", ctypes.c_size_t),
        ("last_active", ctypes.c_int), ("last_factorized", ctypes.c_int),
    ]


_lib = None


def lib():
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(
            f"{LIB_PATH} is missing: build it with python -m paper_1911_10487_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    D = ctypes.c_double
    I = ctypes.c_int
    L.fl_opts_default.argtypes = [ctypes.POINTER(FlOpts)]
    L.fl_opts_default.restype = None
    L.fl_last_error.argtypes = []
    L.fl_last_error.restype = ctypes.c_char_p
    L.fl_plan_create.argtypes = [I, I, I, I, D, ctypes.POINTER(D), ctypes.POINTER(D), D, I,
                                 ctypes.POINTER(FlOpts), ctypes.POINTER(P)]
    L.fl_plan_create.restype = I
    L.fl_invert.argtypes = [P, P, P, D, P]
    L.fl_invert.restype = I
    L.fl_invert_vjp.argtypes = [P, P, P, D, P, P, P]
    L.fl_invert_vjp.restype = I
    L.fl_invert_vjp_noalloc.argtypes = [P, P, P, D, P, P, P]
    L.fl_invert_vjp_noalloc.restype = I
    L.fl_invert_jvp.argtypes = [P, P, P, D, P, P]
    L.fl_invert_jvp.restype = I
    L.fl_forward.argtypes = [P, P, P, D, I, P]
    L.fl_forward.restype = I
    L.fl_plan_info.argtypes = [P, ctypes.POINTER(FlPlanInfo)]
    L.fl_plan_info.restype = I
    L.fl_plan_refresh_info.argtypes = [P]
    L.fl_plan_refresh_info.restype = I
    L.fl_debug_read.argtypes = [P, I, P, ctypes.c_size_t]
    L.fl_debug_read.restype = I
    L.fl_profile_enable.argtypes = [P, I]
    L.fl_profile_enable.restype = I
    L.fl_profile_read.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(I)]
    L.fl_profile_read.restype = I
    L.fl_graph_create.argtypes = [P, P, P, D, P, ctypes.POINTER(P)]
    L.fl_graph_create.restype = I
    L.fl_graph_launch.argtypes = [P]
    L.fl_graph_launch.restype = I
    L.fl_graph_destroy.argtypes = [P]
    L.fl_graph_destroy.restype = None
    PP = ctypes.POINTER(P)
    L.fl_batch_create.argtypes = [PP, I, P, PP]
    L.fl_batch_create.restype = I
    L.fl_batch_invert.argtypes = [P, PP, PP, ctypes.POINTER(D), PP]
    L.fl_batch_invert.restype = I
    L.fl_batch_destroy.argtypes = [P]
    L.fl_batch_destroy.restype = None
    L.fl_plan_destroy.argtypes = [P]
    L.fl_plan_destroy.restype = None
    L.fl_set_frequency_weights.argtypes = [P, ctypes.POINTER(D)]
    L.fl_set_frequency_weights.restype = I
    TP = ctypes.POINTER(FlTuning)
    L.fl_tuning_get.argtypes = [P, TP]
    L.fl_tuning_get.restype = I
    L.fl_tuning_set.argtypes = [P, TP]
    L.fl_tuning_set.restype = I
    L.fl_tuning_variants.argtypes = [P]
    L.fl_tuning_variants.restype = I
    IP = ctypes.POINTER(I)
    L.fl_tuning_describe.argtypes = [P, I, IP, IP, IP]
    L.fl_tuning_describe.restype = I
    L.fl_plan_tune.argtypes = [P, P, P, D, I, P, TP]
    L.fl_plan_tune.restype = I
    _lib = L
    return L


def _check(status):
    if status != FL_OK:
        raise FlError(status, lib().fl_last_error().decode())


def default_opts() -> FlOpts:
    o = FlOpts()
    lib().fl_opts_default(ctypes.byref(o))
    return o


def _stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(name, t, shape, dtypes):
    """Refuse an array that does not match what the kernels will index: a
    wrong shape or dtype would make them read or write past the tensor."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, the plan needs {tuple(shape)}")
    if t.dtype not in dtypes:
        raise ValueError(f"{name} has dtype {t.dtype}, the plan needs one of {dtypes}")


class Plan:
    """A flayer plan for one geometry and frequency set (owns device tables)."""

    def __init__(self, nx, ny, nz, nd, h, planes, omegas, c0=1.0, px=0, py=0, precision=0,
                 tau=1.5, eta=1e-10, combine=0, input_dtype=0, stream=None, max_chunk=0,
                 kernel_mode=0, damping=0.0, alpha_rule=0, factor_per_system=0,
                 forward_method=0, prefactor=0, regularizer=0, hz=0.0):
        o = default_opts()
        o.px, o.py, o.precision = px, py, precision
        o.tau, o.eta, o.combine, o.input_dtype = tau, eta, combine, input_dtype
        o.max_chunk = max_chunk
        o.kernel_mode, o.damping = kernel_mode, damping
        o.alpha_rule, o.factor_per_system = alpha_rule, factor_per_system
        o.forward_method, o.prefactor = forward_method, prefactor
        o.regularizer = regularizer
        o.hz = hz
        o.stream = stream if stream is not None else _stream_handle()
        planes = np.ascontiguousarray(planes, np.float64)
        omegas = np.ascontiguousarray(omegas, np.float64)
        h_ = ctypes.c_void_p()
        _check(lib().fl_plan_create(
            nx, ny, nz, nd, h,
            planes.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            omegas.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            c0, len(omegas), ctypes.byref(o), ctypes.byref(h_)))
        self._h = h_
        self.nx, self.ny, self.nz, self.nd = nx, ny, nz, nd
        self.n_omega = len(omegas)
        self.combine = combine
        self.input_dtype = input_dtype
        info = self.info()
        self.px, self.py = info.px, info.py

    # ---- shapes and dtypes the kernels assume

    def _in_dtypes(self):
        import torch
        return (torch.complex64,) if self.input_dtype == 1 else (torch.complex128,)

    def _w_shape(self):
        return (self.n_omega, self.nd, self.py, self.px)

    def _u_shape(self):
        return (self.n_omega, self.nz, self.ny, self.nx)

    def _xi_shape(self):
        s = (self.nz, self.ny, self.nx)
        return (self.n_omega,) + s if self.combine == 1 else s

    def _check_inputs(self, W, u0):
        _need("W", W, self._w_shape(), self._in_dtypes())
        _need("u0", u0, self._u_shape(), self._in_dtypes())
        if u0.device != W.device:
            raise ValueError("W and u0 must be on the same device")

    @classmethod
    def from_problem(cls, p, **kw):
        if getattr(p, "hz", None) is not None:
            kw.setdefault("hz", p.hz)
        return cls(p.nx, p.ny, p.nz, p.nd, p.h, p.planes, p.omegas, p.c0, p.px, p.py, **kw)

    def info(self) -> FlPlanInfo:
        i = FlPlanInfo()
        _check(lib().fl_plan_info(self._h, ctypes.byref(i)))
        return i

    def active_systems(self) -> int:
        _check(lib().fl_plan_refresh_info(self._h))
        return self.info().last_active

    def set_frequency_weights(self, weights=None):
        """Weights of the frequencies in the least-squares xi (None: all
        ones); a weight of 0 drops that frequency's solve."""
        if weights is None:
            _check(lib().fl_set_frequency_weights(self._h, None))
            return
        w = np.ascontiguousarray(weights, np.float64)
        if w.shape != (self.n_omega,):
            raise ValueError(f"need {self.n_omega} weights")
        _check(lib().fl_set_frequency_weights(
            self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))

    def factorized_systems(self) -> int:
        """Matrices factorized by the last invert (active symmetry orbits
        when factorizations are shared)."""
        _check(lib().fl_plan_refresh_info(self._h))
        return self.info().last_factorized

    def invert(self, W, u0, delta, xi_out=None):
        """W (n_omega, nd, py, px) and u0 (n_omega, nz, ny, nx): complex
        tensors on the GPU. Returns xi (nz, ny, nx) complex128 on the GPU."""
        import torch
        self._check_inputs(W, u0)
        if xi_out is None:
            xi_out = torch.empty(self._xi_shape(), dtype=torch.complex128, device=W.device)
        _need("xi_out", xi_out, self._xi_shape(), (torch.complex128,))
        _check(lib().fl_invert(self._h, ctypes.c_void_p(W.data_ptr()),
                               ctypes.c_void_p(u0.data_ptr()), float(delta),
                               ctypes.c_void_p(xi_out.data_ptr())))
        return xi_out

    def vjp(self, W, u0, delta, grad_xi, want_u0=False, noalloc=False, out=None):
        """Cotangents of W (and u0) for the xi cotangent grad_xi (complex128).
        noalloc: call fl_invert_vjp_noalloc (workspaces in the library's
        static device array; the cotangents go into `out` = (gW, gu0 or
        None) when given, so that the call itself allocates nothing)."""
        import torch
        self._check_inputs(W, u0)
        if out is not None:
            gW, gu = out
            _need("gW", gW, self._w_shape(), (torch.complex128,))
            if gu is not None:
                _need("gu0", gu, self._u_shape(), (torch.complex128,))
        else:
            gW = torch.empty(W.shape, dtype=torch.complex128, device=W.device)
            gu = (torch.empty(self._u_shape(), dtype=torch.complex128,
                              device=W.device) if want_u0 else None)
        if tuple(grad_xi.shape) != self._xi_shape():
            raise ValueError(f"grad_xi has shape {tuple(grad_xi.shape)}, the plan needs "
                             f"{self._xi_shape()}")
        g = grad_xi
        if not (g.is_cuda and g.dtype == torch.complex128 and g.is_contiguous()):
            g = grad_xi.to(W.device, torch.complex128).contiguous()
        fn = lib().fl_invert_vjp_noalloc if noalloc else lib().fl_invert_vjp
        _check(fn(self._h, ctypes.c_void_p(W.data_ptr()),
                                   ctypes.c_void_p(u0.data_ptr()), float(delta),
                                   ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(gW.data_ptr()),
                                   ctypes.c_void_p(gu.data_ptr() if gu is not None else None)))
        return gW, gu

    def jvp(self, W, u0, delta, dW):
        """Tangent of xi for the data tangent dW (same dtype as W)."""
        import torch
        self._check_inputs(W, u0)
        if tuple(dW.shape) != self._w_shape():
            raise ValueError(f"dW has shape {tuple(dW.shape)}, the plan needs {self._w_shape()}")
        out = torch.empty(self._xi_shape(), dtype=torch.complex128, device=W.device)
        d = dW.to(W.device, W.dtype).contiguous()
        _check(lib().fl_invert_jvp(self._h, ctypes.c_void_p(W.data_ptr()),
                                   ctypes.c_void_p(u0.data_ptr()), float(delta),
                                   ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(out.data_ptr())))
        return out

    def forward(self, xi, u0, W_out=None, maxit=0, tol=1e-12):
        """W = omega^2 G * (xi u) on the data planes' torus: Born data
        (u = u0) for maxit = 0, else u from the BiCGSTAB solve of
        u - omega^2 K(xi u) = u0 (relative residual tol)."""
        import torch
        _need("xi", xi, (self.nz, self.ny, self.nx), (torch.float64,))
        _need("u0", u0, self._u_shape(), self._in_dtypes())
        if W_out is None:
            W_out = torch.empty(self._w_shape(), dtype=torch.complex128, device=u0.device)
        _need("W_out", W_out, self._w_shape(), (torch.complex128,))
        _check(lib().fl_forward(self._h, ctypes.c_void_p(xi.data_ptr()),
                                ctypes.c_void_p(u0.data_ptr()), float(tol), int(maxit),
                                ctypes.c_void_p(W_out.data_ptr())))
        return W_out

    # ---- launch schedule and autotuner

    def tuning(self) -> dict:
        t = FlTuning()
        _check(lib().fl_tuning_get(self._h, ctypes.byref(t)))
        return {"bidiag_variant": t.bidiag_variant, "bidiag_grid": t.bidiag_grid,
                "dp_grid": t.dp_grid, "dp_systems_per_wave": t.dp_systems_per_wave}

    def set_tuning(self, bidiag_variant=0, bidiag_grid=0, dp_grid=0, dp_systems_per_wave=0):
        t = FlTuning(bidiag_variant, bidiag_grid, dp_grid, dp_systems_per_wave)
        _check(lib().fl_tuning_set(self._h, ctypes.byref(t)))

    def tuning_variants(self):
        """[(TR, TC, waves per SIMD)] of the bidiagonalization schedules."""
        out = []
        for v in range(lib().fl_tuning_variants(self._h)):
            a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
            _check(lib().fl_tuning_describe(self._h, v, ctypes.byref(a), ctypes.byref(b),
                                            ctypes.byref(c)))
            out.append((a.value, b.value, c.value))
        return out

    def tune(self, W, u0, delta, reps=3, cache_path=None):
        """Run the autotuner on (W, u0, delta) and keep the fastest schedule.
        With cache_path, a JSON file keyed by geometry, precision and device
        is read first (a hit skips the timing) and updated after a search."""
        import json

        import torch
        key = None
        if cache_path is not None:
            i = self.info()
            key = (f"{torch.cuda.get_device_name(W.device)}|n{self.nz}|{self.px}x{self.py}"
                   f"|F{self.n_omega}|p{i.precision}")
            try:
                with open(cache_path) as fh:
                    cache = json.load(fh)
            except (OSError, ValueError):
                cache = {}
            if key in cache:
                self.set_tuning(**cache[key])
                return self.tuning()
        self._check_inputs(W, u0)
        xi = torch.empty(self._xi_shape(), dtype=torch.complex128, device=W.device)
        t = FlTuning()
        _check(lib().fl_plan_tune(self._h, ctypes.c_void_p(W.data_ptr()),
                                  ctypes.c_void_p(u0.data_ptr()), float(delta), int(reps),
                                  ctypes.c_void_p(xi.data_ptr()), ctypes.byref(t)))
        best = self.tuning()
        if key is not None:
            try:
                with open(cache_path) as fh:
                    cache = json.load(fh)
            except (OSError, ValueError):
                cache = {}
            cache[key] = best
            with open(cache_path, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
        return best

    def tap(self, which, dtype, shape):
        out = np.empty(shape, dtype)
        _check(lib().fl_debug_read(self._h, which, out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def profile(self, on=True):
        _check(lib().fl_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """{stage: (ms summed since the last read, launches)}"""
        n = len(STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int * n)()
        _check(lib().fl_profile_read(self._h, ms, cnt))
        return {STAGES[i]: (ms[i], cnt[i]) for i in range(n)}

    def close(self):
        if self._h:
            lib().fl_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A captured fl_invert (fixed pointers and delta), replayed on the
    plan's stream."""

    def __init__(self, plan, W, u0, delta, xi_out):
        import torch
        plan._check_inputs(W, u0)
        _need("xi_out", xi_out, plan._xi_shape(), (torch.complex128,))
        self._keep = (plan, W, u0, xi_out)
        h = ctypes.c_void_p()
        _check(lib().fl_graph_create(plan._h, ctypes.c_void_p(W.data_ptr()),
                                     ctypes.c_void_p(u0.data_ptr()), float(delta),
                                     ctypes.c_void_p(xi_out.data_ptr()), ctypes.byref(h)))
        self._h = h

    def launch(self):
        _check(lib().fl_graph_launch(self._h))

    def close(self):
        if self._h:
            lib().fl_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several plans (uneven grids) inverted together on forked streams."""

    def __init__(self, plans, stream=None):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        st = stream if stream is not None else _stream_handle()
        _check(lib().fl_batch_create(arr, len(self.plans), st, ctypes.byref(h)))
        self._h = h

    def invert(self, Ws, u0s, deltas, xis):
        import torch
        n = len(self.plans)
        if not (len(Ws) == len(u0s) == len(deltas) == len(xis) == n):
            raise ValueError(f"need {n} of each of W, u0, delta and xi")
        for p, W, u0, xi in zip(self.plans, Ws, u0s, xis):
            p._check_inputs(W, u0)
            _need("xi", xi, p._xi_shape(), (torch.complex128,))
        P = ctypes.c_void_p
        W = (P * n)(*[w.data_ptr() for w in Ws])
        U = (P * n)(*[u.data_ptr() for u in u0s])
        X = (P * n)(*[x.data_ptr() for x in xis])
        D = (ctypes.c_double * n)(*[float(d) for d in deltas])
        _check(lib().fl_batch_invert(self._h, W, U, D, X))
        return xis

    def close(self):
        if self._h:
            lib().fl_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
