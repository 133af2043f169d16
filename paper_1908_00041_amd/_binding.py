"""Thin ctypes binding of libvsht.so (include/vsht.h).

Only argument marshalling happens here; every step of the transforms runs in
the HIP kernels.  PyTorch supplies device memory and the current stream.
If the library has not been built, every entry point raises; there is no
fallback implementation.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvsht.so")

VSHT_OK, VSHT_EINVAL, VSHT_ENOWEIGHTS, VSHT_ENOMEM, VSHT_EDEVICE, VSHT_EUNSUPPORTED = range(6)
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
PLAN_RINGS, PLAN_SCATTERED = 0, 1

# every symbol include/vsht.h declares
EXPORTED = ("vsht_num_coeffs", "vsht_plan", "vsht_forward", "vsht_forward_unweighted",
            "vsht_adjoint", "vsht_plan_info", "vsht_plan_destroy", "vsht_status_string",
            "vsht_last_error", "vsht_set_stage_timing", "vsht_get_stage_times",
            "vsht_forward_many", "vsht_adjoint_many")
VSHT_UNIT_WEIGHTS, VSHT_TIMES_WEIGHTS = 1, 2
STAGES = ("ring_fwd", "leg_fwd", "recombine", "prep", "leg_adj", "ring_adj", "scattered")


class vsht_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("device", ctypes.c_int)]


class vsht_plan_info_t(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("precision", ctypes.c_int), ("kind", ctypes.c_int),
                ("n_points", ctypes.c_int64), ("n_rings", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("max_nphi", ctypes.c_int64),
                ("has_weights", ctypes.c_int), ("workspace_bytes", ctypes.c_size_t),
                ("table_bytes", ctypes.c_size_t)]


class VshtError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(message)
        self.status = status


_lib = None


def load_library(path=LIB_PATH):
    """Load libvsht.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libvsht.so not found at %s; build it with "
                          "`python -m paper_1908_00041_amd.build`" % path)
    lib = ctypes.CDLL(path)
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.vsht_num_coeffs.argtypes = [ci]
    lib.vsht_num_coeffs.restype = i64
    lib.vsht_plan.argtypes = [ci, i64, vp, vp, ctypes.POINTER(vsht_opts), ctypes.POINTER(vp)]
    lib.vsht_plan.restype = ci
    for name in ("vsht_forward", "vsht_forward_unweighted"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp, vp]
        getattr(lib, name).restype = ci
    lib.vsht_adjoint.argtypes = [vp, vp, vp, vp, vp]
    lib.vsht_adjoint.restype = ci
    for name in ("vsht_forward_many", "vsht_adjoint_many"):
        getattr(lib, name).argtypes = [vp, i64, vp, vp, vp, ci, vp]
        getattr(lib, name).restype = ci
    lib.vsht_plan_info.argtypes = [vp, ctypes.POINTER(vsht_plan_info_t)]
    lib.vsht_plan_info.restype = ci
    lib.vsht_plan_destroy.argtypes = [vp]
    lib.vsht_plan_destroy.restype = ci
    lib.vsht_status_string.argtypes = [ci]
    lib.vsht_status_string.restype = ctypes.c_char_p
    lib.vsht_last_error.argtypes = []
    lib.vsht_last_error.restype = ctypes.c_char_p
    lib.vsht_set_stage_timing.argtypes = [vp, ci]
    lib.vsht_set_stage_timing.restype = ci
    lib.vsht_get_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64), ci]
    lib.vsht_get_stage_times.restype = ci
    _lib = lib
    return lib


def _raise_for(status, what):
    if status != VSHT_OK:
        lib = load_library()
        raise VshtError(status, "%s: %s (%s)" % (what, lib.vsht_status_string(status).decode(),
                                                 lib.vsht_last_error().decode()))


# ---- the C entry points under their own names (pointers as Python ints) ----
def vsht_num_coeffs(L):
    return load_library().vsht_num_coeffs(int(L))


def vsht_plan(L, n, xyz_ptr, w_ptr, opts, out_handle):
    return load_library().vsht_plan(L, n, xyz_ptr, w_ptr, opts, out_handle)


def vsht_forward(plan, T_ptr, a_ptr, b_ptr, stream):
    return load_library().vsht_forward(plan, T_ptr, a_ptr, b_ptr, stream)


def vsht_forward_unweighted(plan, T_ptr, a_ptr, b_ptr, stream):
    return load_library().vsht_forward_unweighted(plan, T_ptr, a_ptr, b_ptr, stream)


def vsht_adjoint(plan, a_ptr, b_ptr, T_ptr, stream):
    return load_library().vsht_adjoint(plan, a_ptr, b_ptr, T_ptr, stream)


def vsht_forward_many(plan, count, T_ptr, a_ptr, b_ptr, flags, stream):
    return load_library().vsht_forward_many(plan, count, T_ptr, a_ptr, b_ptr, flags, stream)


def vsht_adjoint_many(plan, count, a_ptr, b_ptr, T_ptr, flags, stream):
    return load_library().vsht_adjoint_many(plan, count, a_ptr, b_ptr, T_ptr, flags, stream)


def vsht_plan_info(plan, info):
    return load_library().vsht_plan_info(plan, info)


def vsht_plan_destroy(plan):
    return load_library().vsht_plan_destroy(plan)


# ---- convenience layer on torch tensors ----
def _torch():
    import torch
    return torch


class Plan:
    """A transform plan: bandlimit L, points (n, 3) and optional weights (n,).

    ``forward(T)`` and ``adjoint(a, b)`` take and return torch tensors on the
    plan's GPU (complex128 for precision 'fp64', complex64 otherwise) and run
    on the current torch stream.
    """

    def __init__(self, L, points, weights=None, precision="fp64", device=None):
        torch = _torch()
        lib = load_library()
        if precision not in PRECISIONS:
            raise ValueError("precision must be one of %s" % sorted(PRECISIONS))
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        n = pts.shape[0]
        w = None
        if weights is not None:
            w = np.ascontiguousarray(weights, dtype=np.float64).reshape(-1)
            if w.shape[0] != n:
                raise ValueError("weights must have one entry per point")
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", int(device))
        self.L = int(L)
        self.n = n
        self.precision = precision
        self.dtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.K = int(lib.vsht_num_coeffs(self.L))
        opts = vsht_opts(PRECISIONS[precision], int(device))
        h = ctypes.c_void_p()
        st = lib.vsht_plan(self.L, n, pts.ctypes.data_as(ctypes.c_void_p),
                           None if w is None else w.ctypes.data_as(ctypes.c_void_p),
                           ctypes.byref(opts), ctypes.byref(h))
        _raise_for(st, "vsht_plan")
        self._h = h
        self._info = self.info()

    def info(self):
        inf = vsht_plan_info_t()
        _raise_for(load_library().vsht_plan_info(self._h, ctypes.byref(inf)), "vsht_plan_info")
        return {f: getattr(inf, f) for f, _ in vsht_plan_info_t._fields_}

    @property
    def kind(self):
        return "rings" if self._info["kind"] == PLAN_RINGS else "scattered"

    def _stream(self):
        return _torch().cuda.current_stream(self.device).cuda_stream

    def _check(self, t, shape, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.device != self.device or t.dtype != self.dtype or tuple(t.shape) != shape:
            raise ValueError("%s must be a %s tensor of shape %s on %s (got %s %s on %s)" % (
                name, self.dtype, shape, self.device, t.dtype, tuple(t.shape), t.device))
        return t.contiguous()

    def forward(self, T, a=None, b=None, weighted=True):
        torch = _torch()
        T = self._check(T, (self.n, 3), "T")
        if a is None:
            a = torch.empty(self.K, dtype=self.dtype, device=self.device)
        if b is None:
            b = torch.empty(self.K, dtype=self.dtype, device=self.device)
        fn = vsht_forward if weighted else vsht_forward_unweighted
        _raise_for(fn(self._h, T.data_ptr(), a.data_ptr(), b.data_ptr(), self._stream()),
                   "vsht_forward" if weighted else "vsht_forward_unweighted")
        return a, b

    def forward_unweighted(self, T, a=None, b=None):
        return self.forward(T, a, b, weighted=False)

    def adjoint(self, a, b, T=None):
        torch = _torch()
        a = self._check(a, (self.K,), "a")
        b = self._check(b, (self.K,), "b")
        if T is None:
            T = torch.empty((self.n, 3), dtype=self.dtype, device=self.device)
        _raise_for(vsht_adjoint(self._h, a.data_ptr(), b.data_ptr(), T.data_ptr(), self._stream()),
                   "vsht_adjoint")
        return T

    def _check_batch(self, t, tail, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.device != self.device or t.dtype != self.dtype or tuple(t.shape[t.dim() - len(tail):]) != tail \
                or t.dim() < len(tail):
            raise ValueError("%s must be a %s tensor of shape (..., %s) on %s (got %s %s on %s)" % (
                name, self.dtype, ", ".join(map(str, tail)), self.device, t.dtype, tuple(t.shape), t.device))
        return t.contiguous()

    def forward_many(self, T, unit_weights=False):
        """Forward transform of every field of T (..., n, 3) -> a, b (..., K)."""
        torch = _torch()
        T = self._check_batch(T, (self.n, 3), "T")
        lead = tuple(T.shape[:-2])
        count = int(np.prod(lead)) if lead else 1
        a = torch.empty(lead + (self.K,), dtype=self.dtype, device=self.device)
        b = torch.empty_like(a)
        _raise_for(vsht_forward_many(self._h, count, T.data_ptr(), a.data_ptr(), b.data_ptr(),
                                     VSHT_UNIT_WEIGHTS if unit_weights else 0, self._stream()),
                   "vsht_forward_many")
        return a, b

    def adjoint_many(self, a, b, times_weights=False):
        """Adjoint transform of every coefficient block a, b (..., K) -> T (..., n, 3)."""
        torch = _torch()
        a = self._check_batch(a, (self.K,), "a")
        b = self._check_batch(b, (self.K,), "b")
        if a.shape != b.shape:
            raise ValueError("a and b must have the same shape")
        lead = tuple(a.shape[:-1])
        count = int(np.prod(lead)) if lead else 1
        T = torch.empty(lead + (self.n, 3), dtype=self.dtype, device=self.device)
        _raise_for(vsht_adjoint_many(self._h, count, a.data_ptr(), b.data_ptr(), T.data_ptr(),
                                     VSHT_TIMES_WEIGHTS if times_weights else 0, self._stream()),
                   "vsht_adjoint_many")
        return T

    def set_stage_timing(self, enable):
        _raise_for(load_library().vsht_set_stage_timing(self._h, 1 if enable else 0),
                   "vsht_set_stage_timing")

    def stage_times(self):
        """{stage: (total_ms, launches)} recorded since the previous read."""
        n = len(STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        _raise_for(load_library().vsht_get_stage_times(self._h, ms, cnt, n), "vsht_get_stage_times")
        return {STAGES[i]: (ms[i], cnt[i]) for i in range(n)}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().vsht_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
