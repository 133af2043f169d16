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
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
PLAN_RINGS, PLAN_SCATTERED, PLAN_BATCH = 0, 1, 2

# every symbol include/vsht.h declares
EXPORTED = ("vsht_num_coeffs", "vsht_plan", "vsht_forward", "vsht_forward_unweighted",
            "vsht_adjoint", "vsht_plan_info", "vsht_plan_destroy", "vsht_status_string",
            "vsht_last_error", "vsht_set_stage_timing", "vsht_get_stage_times",
            "vsht_forward_many", "vsht_adjoint_many", "vsht_plan_batch", "vsht_batch_adjoint",
            "vsht_batch_forward", "vsht_batch_roundtrip", "vsht_batch_set_config",
            "vsht_batch_get_config", "vsht_batch_autotune", "vsht_batch_field_times",
            "vsht_num_sht_coeffs", "vsht_sht_forward", "vsht_sht_adjoint", "vsht_forward_static",
            "vsht_workspace_bytes")
VSHT_UNIT_WEIGHTS, VSHT_TIMES_WEIGHTS = 1, 2
STAGES = ("ring_fwd", "leg_fwd", "recombine", "prep", "leg_adj", "ring_adj", "scattered")


class vsht_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("device", ctypes.c_int), ("flags", ctypes.c_int),
                ("nfft_eps", ctypes.c_double), ("tune_cache", ctypes.c_char_p)]


VSHT_OPT_SCATTERED_DIRECT = 1
VSHT_OPT_NO_FOLD = 2


class vsht_plan_info_t(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int), ("precision", ctypes.c_int), ("kind", ctypes.c_int),
                ("n_points", ctypes.c_int64), ("n_rings", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("max_nphi", ctypes.c_int64),
                ("has_weights", ctypes.c_int), ("workspace_bytes", ctypes.c_size_t),
                ("table_bytes", ctypes.c_size_t), ("nfft_grid", ctypes.c_int64)]


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
    for name in ("vsht_forward", "vsht_forward_unweighted", "vsht_forward_static"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp, vp]
        getattr(lib, name).restype = ci
    lib.vsht_adjoint.argtypes = [vp, vp, vp, vp, vp]
    lib.vsht_adjoint.restype = ci
    lib.vsht_num_sht_coeffs.argtypes = [ci]
    lib.vsht_num_sht_coeffs.restype = i64
    for name in ("vsht_sht_forward", "vsht_sht_adjoint"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp]
        getattr(lib, name).restype = ci
    for name in ("vsht_forward_many", "vsht_adjoint_many"):
        getattr(lib, name).argtypes = [vp, i64, vp, vp, vp, ci, vp]
        getattr(lib, name).restype = ci
    pp = ctypes.POINTER(ctypes.c_void_p)
    pd = ctypes.POINTER(ctypes.c_double)
    pi = ctypes.POINTER(ctypes.c_int)
    lib.vsht_plan_batch.argtypes = [ci, pi, ctypes.POINTER(i64), pp, pp, ctypes.POINTER(vsht_opts),
                                    ctypes.POINTER(vp)]
    lib.vsht_plan_batch.restype = ci
    for name in ("vsht_batch_adjoint", "vsht_batch_forward"):
        getattr(lib, name).argtypes = [vp, pp, pp, pp, vp]
        getattr(lib, name).restype = ci
    lib.vsht_batch_roundtrip.argtypes = [vp, pp, pp, pp, pp, pp, vp]
    lib.vsht_batch_roundtrip.restype = ci
    lib.vsht_batch_set_config.argtypes = [vp, ci, ci, ci, ci, ci]
    lib.vsht_batch_set_config.restype = ci
    lib.vsht_batch_get_config.argtypes = [vp, pi, pi, pi, pi, pi]
    lib.vsht_batch_get_config.restype = ci
    lib.vsht_batch_autotune.argtypes = [vp, pp, pp, pp, pp, pp, ci, pd, vp]
    lib.vsht_batch_autotune.restype = ci
    lib.vsht_batch_field_times.argtypes = [vp, pd, pd]
    lib.vsht_batch_field_times.restype = ci
    lib.vsht_plan_info.argtypes = [vp, ctypes.POINTER(vsht_plan_info_t)]
    lib.vsht_plan_info.restype = ci
    lib.vsht_workspace_bytes.argtypes = [vp]
    lib.vsht_workspace_bytes.restype = ctypes.c_size_t
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


def vsht_forward_static(plan, T_ptr, a_ptr, b_ptr, stream):
    return load_library().vsht_forward_static(plan, T_ptr, a_ptr, b_ptr, stream)


def vsht_adjoint(plan, a_ptr, b_ptr, T_ptr, stream):
    return load_library().vsht_adjoint(plan, a_ptr, b_ptr, T_ptr, stream)


def vsht_num_sht_coeffs(L):
    return load_library().vsht_num_sht_coeffs(L)


def vsht_sht_forward(plan, f_ptr, flm_ptr, stream):
    return load_library().vsht_sht_forward(plan, f_ptr, flm_ptr, stream)


def vsht_sht_adjoint(plan, flm_ptr, f_ptr, stream):
    return load_library().vsht_sht_adjoint(plan, flm_ptr, f_ptr, stream)


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

    def __init__(self, L, points, weights=None, precision="fp64", device=None, scattered="grid",
                 nfft_eps=0.0, fold=True):
        torch = _torch()
        if scattered not in ("grid", "direct"):
            raise ValueError("scattered must be 'grid' or 'direct'")
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
        flags = (VSHT_OPT_SCATTERED_DIRECT if scattered == "direct" else 0) | (0 if fold else VSHT_OPT_NO_FOLD)
        opts = vsht_opts(PRECISIONS[precision], int(device), flags, float(nfft_eps), None)
        h = ctypes.c_void_p()
        st = lib.vsht_plan(self.L, n, pts.ctypes.data_as(ctypes.c_void_p),
                           None if w is None else w.ctypes.data_as(ctypes.c_void_p),
                           ctypes.byref(opts), ctypes.byref(h))
        _raise_for(st, "vsht_plan")
        self._h = h
        self._info = self.info()

    def workspace_bytes(self):
        """Device workspace the plan owns (bytes)."""
        return int(load_library().vsht_workspace_bytes(self._h))

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
        """An input: right dtype, shape and device; a contiguous copy if it is a view."""
        torch = _torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a torch tensor" % name)
        if t.device != self.device or t.dtype != self.dtype or tuple(t.shape) != shape:
            raise ValueError("%s must be a %s tensor of shape %s on %s (got %s %s on %s)" % (
                name, self.dtype, shape, self.device, t.dtype, tuple(t.shape), t.device))
        return t.contiguous()

    def _out(self, t, shape, name):
        """An output: allocated when None, else checked like an input and required to be
        contiguous (the kernels write through its pointer; a copy would lose the results)."""
        torch = _torch()
        if t is None:
            return torch.empty(shape, dtype=self.dtype, device=self.device)
        t2 = self._check(t, shape, name)
        if t2.data_ptr() != t.data_ptr() or not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
        return t

    def forward(self, T, a=None, b=None, weighted=True):
        T = self._check(T, (self.n, 3), "T")
        a = self._out(a, (self.K,), "a")
        b = self._out(b, (self.K,), "b")
        fn = vsht_forward if weighted else vsht_forward_unweighted
        _raise_for(fn(self._h, T.data_ptr(), a.data_ptr(), b.data_ptr(), self._stream()),
                   "vsht_forward" if weighted else "vsht_forward_unweighted")
        return a, b

    def forward_unweighted(self, T, a=None, b=None):
        return self.forward(T, a, b, weighted=False)

    def adjoint(self, a, b, T=None):
        a = self._check(a, (self.K,), "a")
        b = self._check(b, (self.K,), "b")
        T = self._out(T, (self.n, 3), "T")
        _raise_for(vsht_adjoint(self._h, a.data_ptr(), b.data_ptr(), T.data_ptr(), self._stream()),
                   "vsht_adjoint")
        return T

    def sht_forward(self, f, flm=None):
        """Scalar forward transform (ring plans with weights): f (n,) -> flm ((L+1)^2,)."""
        f = self._check(f, (self.n,), "f")
        flm = self._out(flm, (vsht_num_sht_coeffs(self.L),), "flm")
        _raise_for(vsht_sht_forward(self._h, f.data_ptr(), flm.data_ptr(), self._stream()),
                   "vsht_sht_forward")
        return flm

    def sht_adjoint(self, flm, f=None):
        """Scalar adjoint transform (ring plans): flm ((L+1)^2,) -> f (n,)."""
        flm = self._check(flm, (vsht_num_sht_coeffs(self.L),), "flm")
        f = self._out(f, (self.n,), "f")
        _raise_for(vsht_sht_adjoint(self._h, flm.data_ptr(), f.data_ptr(), self._stream()),
                   "vsht_sht_adjoint")
        return f

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


def _ptr_array(tensors):
    return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])


class BatchPlan:
    """Many independent fields, field f with bandlimit Ls[f] on its own ring grid
    grids[f] = (points (n_f, 3), weights (n_f,)); one precision for all.

    Each call runs every stage as one launch over all fields, replayed from a
    HIP graph on the current torch stream.  Tensors are lists with one entry
    per field (complex128 for 'fp64', complex64 otherwise).
    """

    def __init__(self, Ls, grids, precision="fp64", device=None, tune_cache=None):
        torch = _torch()
        lib = load_library()
        if precision not in PRECISIONS:
            raise ValueError("precision must be one of %s" % sorted(PRECISIONS))
        F = len(Ls)
        if F != len(grids) or F == 0:
            raise ValueError("need one grid per bandlimit")
        pts = [np.ascontiguousarray(g[0], dtype=np.float64).reshape(-1, 3) for g in grids]
        wts = [np.ascontiguousarray(g[1], dtype=np.float64).reshape(-1) for g in grids]
        for p_, w_ in zip(pts, wts):
            if len(p_) != len(w_):
                raise ValueError("weights must have one entry per point")
        if device is None:
            device = torch.cuda.current_device()
        self.device = torch.device("cuda", int(device))
        self.precision = precision
        self.dtype = torch.complex128 if precision == "fp64" else torch.complex64
        self.Ls = [int(L) for L in Ls]
        self.ns = [len(p_) for p_ in pts]
        self.Ks = [int(lib.vsht_num_coeffs(L)) for L in self.Ls]
        Larr = (ctypes.c_int * F)(*self.Ls)
        narr = (ctypes.c_int64 * F)(*self.ns)
        xarr = (ctypes.c_void_p * F)(*[p_.ctypes.data for p_ in pts])
        warr = (ctypes.c_void_p * F)(*[w_.ctypes.data for w_ in wts])
        self._tune_cache = None if tune_cache is None else os.fsencode(tune_cache)
        opts = vsht_opts(PRECISIONS[precision], int(device), 0, 0.0, self._tune_cache)
        h = ctypes.c_void_p()
        st = lib.vsht_plan_batch(F, Larr, narr, xarr, warr, ctypes.byref(opts), ctypes.byref(h))
        _raise_for(st, "vsht_plan_batch")
        self._h = h

    def __len__(self):
        return len(self.Ls)

    def _stream(self):
        return _torch().cuda.current_stream(self.device).cuda_stream

    def _check(self, ts, shapes, name, output=False):
        """Inputs: right dtype, shape and device (views are copied).  Outputs: the same,
        and contiguous (the kernels write through the pointers)."""
        torch = _torch()
        if len(ts) != len(self.Ls):
            raise ValueError("%s: need one tensor per field" % name)
        out = []
        for t, shp in zip(ts, shapes):
            if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != self.dtype \
                    or tuple(t.shape) != shp:
                raise ValueError("%s: every entry must be a %s tensor on %s of its field's shape"
                                 % (name, self.dtype, self.device))
            if output and not t.is_contiguous():
                raise ValueError("%s: output tensors must be contiguous" % name)
            out.append(t if output else t.contiguous())
        return out

    def empty_coeffs(self):
        torch = _torch()
        return [torch.empty(K, dtype=self.dtype, device=self.device) for K in self.Ks]

    def empty_fields(self):
        torch = _torch()
        return [torch.empty((n, 3), dtype=self.dtype, device=self.device) for n in self.ns]

    def adjoint(self, a, b, T=None):
        cs = [(K,) for K in self.Ks]
        a, b = self._check(a, cs, "a"), self._check(b, cs, "b")
        T = self.empty_fields() if T is None else self._check(T, [(n, 3) for n in self.ns], "T", True)
        self._keep = (a, b, T)
        _raise_for(load_library().vsht_batch_adjoint(self._h, _ptr_array(a), _ptr_array(b), _ptr_array(T),
                                                     self._stream()), "vsht_batch_adjoint")
        return T

    def forward(self, T, a=None, b=None):
        T = self._check(T, [(n, 3) for n in self.ns], "T")
        a = self.empty_coeffs() if a is None else self._check(a, [(K,) for K in self.Ks], "a", True)
        b = self.empty_coeffs() if b is None else self._check(b, [(K,) for K in self.Ks], "b", True)
        self._keep = (T, a, b)
        _raise_for(load_library().vsht_batch_forward(self._h, _ptr_array(T), _ptr_array(a), _ptr_array(b),
                                                     self._stream()), "vsht_batch_forward")
        return a, b

    def _rt_args(self, a, b, T, a2, b2):
        cs = [(K,) for K in self.Ks]
        a, b = self._check(a, cs, "a"), self._check(b, cs, "b")
        T = self.empty_fields() if T is None else self._check(T, [(n, 3) for n in self.ns], "T", True)
        a2 = self.empty_coeffs() if a2 is None else self._check(a2, cs, "a2", True)
        b2 = self.empty_coeffs() if b2 is None else self._check(b2, cs, "b2", True)
        return a, b, T, a2, b2

    def roundtrip(self, a, b, T=None, a2=None, b2=None):
        """Adjoint a, b -> T, then forward T -> a2, b2, as one graph replay."""
        a, b, T, a2, b2 = self._rt_args(a, b, T, a2, b2)
        self._keep = (a, b, T, a2, b2)
        _raise_for(load_library().vsht_batch_roundtrip(
            self._h, _ptr_array(a), _ptr_array(b), _ptr_array(T), _ptr_array(a2), _ptr_array(b2),
            self._stream()), "vsht_batch_roundtrip")
        return T, a2, b2

    def autotune(self, a, b, T=None, a2=None, b2=None, reps=3):
        """Time every launch shape on these buffers, keep the fastest; returns its ms per roundtrip."""
        a, b, T, a2, b2 = self._rt_args(a, b, T, a2, b2)
        self._keep = (a, b, T, a2, b2)
        best = ctypes.c_double()
        _raise_for(load_library().vsht_batch_autotune(
            self._h, _ptr_array(a), _ptr_array(b), _ptr_array(T), _ptr_array(a2), _ptr_array(b2),
            int(reps), ctypes.byref(best), self._stream()), "vsht_batch_autotune")
        return best.value

    def config(self):
        x, y, z, r, c = (ctypes.c_int() for _ in range(5))
        _raise_for(load_library().vsht_batch_get_config(self._h, ctypes.byref(x), ctypes.byref(y),
                                                        ctypes.byref(z), ctypes.byref(r), ctypes.byref(c)),
                   "vsht_batch_get_config")
        return {"adj_nw": x.value, "fwd_merge": y.value, "lpt": z.value, "ring_nt": r.value,
                "chains": c.value}

    def set_config(self, adj_nw=4, fwd_merge=0, lpt=1, ring_nt=256, chains=0):
        _raise_for(load_library().vsht_batch_set_config(self._h, int(adj_nw), int(fwd_merge), int(lpt),
                                                        int(ring_nt), int(chains)), "vsht_batch_set_config")

    def field_times(self):
        """(start_us, end_us) per field of the last call, device wall clock."""
        F = len(self.Ls)
        t0 = (ctypes.c_double * F)()
        t1 = (ctypes.c_double * F)()
        _raise_for(load_library().vsht_batch_field_times(self._h, t0, t1), "vsht_batch_field_times")
        return np.array(t0[:]), np.array(t1[:])

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().vsht_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
