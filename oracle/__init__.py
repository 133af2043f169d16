"""CPU FP64 oracle for the forward and adjoint vector spherical harmonic
transforms (FaVeST).  TEST INFRASTRUCTURE ONLY: the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may use it; the library never
does.  It shares no code with the HIP path.

The arithmetic lives in ``vsht_oracle.c`` (plain C, binary64, OpenMP, built
with ``-ffp-contract=off``); this module only builds it and marshals numpy
arrays.  What each entry point computes, with the paper passage it follows:

* :func:`sph_harm`   scalar harmonics Y_{l,m} (Section 3).
* :func:`vsh`        Y^div, Y^curl of Definition 3.1 via eq. (Blm1), (Blm2),
                     (ninecoeff), (vsh2).
* :func:`forward`    Definition 4.1, eq. (fwdvsht2).
* :func:`adjoint`    Definition 4.2, eq. (SLvec).
* :func:`forward_subset`  eq. (fwdvsht2) for chosen coefficient indices.

Coefficient order: index j = l*l + l + m - 1 for 1 <= l <= L, |m| <= l.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vsht_oracle.c")
_LIB = os.path.join(_HERE, "libvsht_oracle.so")
_lib = None


def build(force=True):
    """Compile the oracle with gcc (binary64, no FMA contraction, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, i32, dp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        lib.vo_num_threads.restype = i32
        lib.vo_sph_harm.argtypes = [i32, i64, dp, dp]
        lib.vo_vsh.argtypes = [i32, i64, dp, dp, dp]
        lib.vo_forward.argtypes = [i32, i64, dp, dp, dp, dp, dp]
        lib.vo_adjoint.argtypes = [i32, dp, dp, i64, dp, dp]
        lib.vo_forward_subset.argtypes = [i32, i64, dp, dp, dp, i64, dp, dp, dp]
        for f in (lib.vo_sph_harm, lib.vo_vsh, lib.vo_forward, lib.vo_adjoint, lib.vo_forward_subset):
            f.restype = None
        _lib = lib
    return _lib


def _f64(x, shape=None):
    a = np.ascontiguousarray(x, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _c128(x):
    return np.ascontiguousarray(x, dtype=np.complex128)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_coeffs(L):
    return L * (L + 2)


def num_threads():
    return _load().vo_num_threads()


def sph_harm(Lmax, xyz):
    """Y_{l,m}(x_k), 0 <= l <= Lmax, as (n, (Lmax+1)^2) complex, index l*l+l+m."""
    xyz = _f64(xyz).reshape(-1, 3)
    n = xyz.shape[0]
    out = np.zeros((n, (Lmax + 1) ** 2), np.complex128)
    _load().vo_sph_harm(Lmax, n, _ptr(xyz), _ptr(out))
    return out


def vsh(L, xyz):
    """(Y^div, Y^curl) at the points, each (n, L(L+2), 3) complex."""
    xyz = _f64(xyz).reshape(-1, 3)
    n = xyz.shape[0]
    K = num_coeffs(L)
    d = np.zeros((n, K, 3), np.complex128)
    c = np.zeros((n, K, 3), np.complex128)
    _load().vo_vsh(L, n, _ptr(xyz), _ptr(d), _ptr(c))
    return d, c


def forward(L, xyz, w, T):
    """eq. (fwdvsht2): a_j = sum_k w_k Y^div_j(x_k)^* T_k, b_j with Y^curl."""
    xyz = _f64(xyz).reshape(-1, 3)
    n = xyz.shape[0]
    w = _f64(w).reshape(n)
    T = _c128(T).reshape(n, 3)
    K = num_coeffs(L)
    a = np.zeros(K, np.complex128)
    b = np.zeros(K, np.complex128)
    _load().vo_forward(L, n, _ptr(xyz), _ptr(w), _ptr(T), _ptr(a), _ptr(b))
    return a, b


def adjoint(L, a, b, xyz):
    """eq. (SLvec): T(x_k) = sum_j a_j Y^div_j(x_k) + b_j Y^curl_j(x_k), (n, 3)."""
    K = num_coeffs(L)
    a = _c128(a).reshape(K)
    b = _c128(b).reshape(K)
    xyz = _f64(xyz).reshape(-1, 3)
    n = xyz.shape[0]
    T = np.zeros((n, 3), np.complex128)
    _load().vo_adjoint(L, _ptr(a), _ptr(b), n, _ptr(xyz), _ptr(T))
    return T


def forward_subset(L, xyz, w, T, coef_index):
    """eq. (fwdvsht2) for the coefficient indices given (each in [0, L(L+2)))."""
    xyz = _f64(xyz).reshape(-1, 3)
    n = xyz.shape[0]
    w = _f64(w).reshape(n)
    T = _c128(T).reshape(n, 3)
    idx = np.ascontiguousarray(coef_index, dtype=np.int64).reshape(-1)
    K = num_coeffs(L)
    if idx.size and (idx.min() < 0 or idx.max() >= K):
        raise ValueError("coefficient index out of range")
    a = np.zeros(idx.size, np.complex128)
    b = np.zeros(idx.size, np.complex128)
    _load().vo_forward_subset(L, n, _ptr(xyz), _ptr(w), _ptr(T), idx.size, _ptr(idx),
                              _ptr(a), _ptr(b))
    return a, b
