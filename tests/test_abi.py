"""CPU checks of the C interface: the library loads, exports every function
include/vsht.h declares, and rejects invalid arguments before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1908_00041_amd as v
from paper_1908_00041_amd import _binding as B
import vsht_inputs as vi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "vsht.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vsht_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = v.load_library()
    names = declared_functions()
    assert names, "no declarations parsed"
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(B.EXPORTED) == names


def test_num_sht_coeffs():
    lib = B.load_library()
    assert [lib.vsht_num_sht_coeffs(L) for L in (-1, 0, 1, 2, 1024)] == [0, 1, 4, 9, 1025 ** 2]


def test_num_coeffs():
    for L, K in [(0, 0), (-3, 0), (1, 3), (16, 288), (1024, 1050624)]:
        assert v.vsht_num_coeffs(L) == K


def _plan(L, xyz, w=None, opts=None):
    lib = v.load_library()
    h = ctypes.c_void_p()
    xyz = None if xyz is None else np.ascontiguousarray(xyz, np.float64)
    w = None if w is None else np.ascontiguousarray(w, np.float64)
    n = 0 if xyz is None else len(xyz)
    st = lib.vsht_plan(L, n if xyz is not None else 5,
                       None if xyz is None else xyz.ctypes.data_as(ctypes.c_void_p),
                       None if w is None else w.ctypes.data_as(ctypes.c_void_p),
                       opts, ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("case", ["L0", "n0", "null_xyz", "non_unit", "nan", "one_point_weights",
                                  "bad_precision"])
def test_plan_rejects_invalid(case):
    lib = v.load_library()
    xyz = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    w = np.ones(3)
    opts = None
    if case == "L0":
        st, h = _plan(0, xyz, w)
    elif case == "n0":
        h = ctypes.c_void_p()
        st = lib.vsht_plan(4, 0, xyz.ctypes.data_as(ctypes.c_void_p), None, None, ctypes.byref(h))
    elif case == "null_xyz":
        st, h = _plan(4, None)
    elif case == "non_unit":
        st, h = _plan(4, xyz * 1.001, w)
    elif case == "nan":
        bad = xyz.copy()
        bad[1, 2] = np.nan
        st, h = _plan(4, bad, w)
    elif case == "one_point_weights":
        st, h = _plan(4, xyz[:1], w[:1])
    else:
        st, h = _plan(4, xyz, w, ctypes.byref(B.vsht_opts(7, -1)))
    assert st == B.VSHT_EINVAL
    assert not h.value
    assert len(lib.vsht_last_error()) > 0


def test_plan_rejects_bandlimit_beyond_limit():
    """Plans above L = 4096 are refused before any device work (host check)."""
    lib = B.load_library()
    xyz, _ = vi.uniform_points(16, 5)
    xyz = np.ascontiguousarray(xyz, np.float64)
    h = ctypes.c_void_p()
    st = lib.vsht_plan(4097, len(xyz), xyz.ctypes.data_as(ctypes.c_void_p), None, None, ctypes.byref(h))
    assert st == B.VSHT_EUNSUPPORTED and not h.value
    assert "4096" in B.load_library().vsht_last_error().decode()


def test_null_arguments():
    lib = v.load_library()
    assert lib.vsht_forward(None, None, None, None, None) == B.VSHT_EINVAL
    assert lib.vsht_adjoint(None, None, None, None, None) == B.VSHT_EINVAL
    assert lib.vsht_forward_unweighted(None, None, None, None, None) == B.VSHT_EINVAL
    assert lib.vsht_sht_forward(None, None, None, None) == B.VSHT_EINVAL
    assert lib.vsht_sht_adjoint(None, None, None, None) == B.VSHT_EINVAL
    assert lib.vsht_plan_info(None, None) == B.VSHT_EINVAL
    assert lib.vsht_plan_destroy(None) == B.VSHT_OK
    h = ctypes.c_void_p()
    assert lib.vsht_plan(4, 3, None, None, None, None) == B.VSHT_EINVAL


def test_status_strings():
    lib = v.load_library()
    for s in range(6):
        assert lib.vsht_status_string(s).decode().startswith("VSHT_")


def test_many_null_arguments():
    lib = v.load_library()
    assert lib.vsht_forward_many(None, 1, None, None, None, 0, None) == B.VSHT_EINVAL
    assert lib.vsht_adjoint_many(None, 1, None, None, None, 0, None) == B.VSHT_EINVAL
    assert b"NULL" in lib.vsht_last_error()


def test_batch_plan_rejects_invalid():
    """vsht_plan_batch validates every field before any device work."""
    lib = v.load_library()
    xyz = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    w = np.ones(3)
    h = ctypes.c_void_p()
    L = (ctypes.c_int * 2)(4, 4)
    n = (ctypes.c_int64 * 2)(3, 3)
    X = (ctypes.c_void_p * 2)(xyz.ctypes.data, xyz.ctypes.data)
    W = (ctypes.c_void_p * 2)(w.ctypes.data, w.ctypes.data)
    assert lib.vsht_plan_batch(0, L, n, X, W, None, ctypes.byref(h)) == B.VSHT_EINVAL
    assert lib.vsht_plan_batch(2, None, n, X, W, None, ctypes.byref(h)) == B.VSHT_EINVAL
    Wnull = (ctypes.c_void_p * 2)(w.ctypes.data, None)
    assert lib.vsht_plan_batch(2, L, n, X, Wnull, None, ctypes.byref(h)) == B.VSHT_EINVAL
    assert b"field 1" in lib.vsht_last_error()
    bad = xyz * 2.0
    Xbad = (ctypes.c_void_p * 2)(xyz.ctypes.data, bad.ctypes.data)
    assert lib.vsht_plan_batch(2, L, n, Xbad, W, None, ctypes.byref(h)) == B.VSHT_EINVAL
    assert b"field 1" in lib.vsht_last_error()
    assert not h.value


def test_batch_calls_reject_null_plan():
    lib = v.load_library()
    assert lib.vsht_batch_roundtrip(None, None, None, None, None, None, None) == B.VSHT_EINVAL
    assert lib.vsht_batch_adjoint(None, None, None, None, None) == B.VSHT_EINVAL
    assert lib.vsht_batch_forward(None, None, None, None, None) == B.VSHT_EINVAL
    assert lib.vsht_batch_set_config(None, 4, 0, 1, 256, 1) == B.VSHT_EINVAL
    assert lib.vsht_batch_field_times(None, None, None) == B.VSHT_EINVAL


def _shell_plan(precision="fp64"):
    """A Plan object without a native handle: the binding's argument checks run in
    Python before any C call, so they can be exercised on the CPU."""
    import torch
    p = B.Plan.__new__(B.Plan)
    p.device = torch.device("cpu")
    p.L, p.n, p.K = 4, 10, 24
    p.precision = precision
    p.dtype = torch.complex128 if precision == "fp64" else torch.complex64
    p._h = None
    return p


@pytest.mark.parametrize("case", ["short_a", "dtype_b", "noncontig_T", "short_T", "dtype_flm"])
def test_binding_rejects_bad_outputs(case):
    """Caller-supplied output tensors are checked (shape, dtype, device, contiguity)
    before the library is called; a bad one raises instead of being written past its end
    or into a temporary copy."""
    import torch
    p = _shell_plan()
    c = lambda *s: torch.zeros(s, dtype=torch.complex128)
    T, a, b = c(10, 3), c(24), c(24)
    with pytest.raises(ValueError):
        if case == "short_a":
            p.forward(T, a=c(23), b=b)
        elif case == "dtype_b":
            p.forward(T, a=a, b=torch.zeros(24, dtype=torch.complex64))
        elif case == "noncontig_T":
            p.adjoint(a, b, T=c(3, 10).t())
        elif case == "short_T":
            p.adjoint(a, b, T=c(9, 3))
        else:
            p.sht_forward(torch.zeros(10, dtype=torch.complex128), flm=c(24))


def test_binding_rejects_bad_batch_outputs():
    import torch
    bp = B.BatchPlan.__new__(B.BatchPlan)
    bp.device = torch.device("cpu")
    bp.dtype = torch.complex64
    bp.Ls, bp.ns, bp.Ks = [4], [10], [24]
    bp._h = None
    a = [torch.zeros(24, dtype=torch.complex64)]
    with pytest.raises(ValueError):
        bp.adjoint(a, a, T=[torch.zeros(3, 10, dtype=torch.complex64).t()])
    with pytest.raises(ValueError):
        bp.forward([torch.zeros(10, 3, dtype=torch.complex64)], a=[torch.zeros(23, dtype=torch.complex64)])


def test_opts_checked_on_host():
    """nfft_eps outside [0, 1) and unknown flags are refused before any device work;
    vsht_workspace_bytes(NULL) is 0."""
    lib = B.load_library()
    xyz, _ = vi.uniform_points(16, 5)
    xyz = np.ascontiguousarray(xyz, np.float64)
    h = ctypes.c_void_p()
    for opts in (B.vsht_opts(0, -1, 0, 1.5, None), B.vsht_opts(0, -1, 0, -1e-3, None),
                 B.vsht_opts(0, -1, 0, float("nan"), None), B.vsht_opts(0, -1, 8, 0.0, None)):
        st = lib.vsht_plan(8, len(xyz), xyz.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(opts),
                           ctypes.byref(h))
        assert st == B.VSHT_EINVAL and not h.value
    assert lib.vsht_workspace_bytes(None) == 0
    # the C layout: three ints, the double at offset 16, the pointer at 24
    assert ctypes.sizeof(B.vsht_opts) == 32
    assert B.vsht_opts.nfft_eps.offset == 16 and B.vsht_opts.tune_cache.offset == 24
