"""Planted mistakes in the oracle (on the CPU only): each mutant is a copy of
oracle/vsht_oracle.c with one plausible error, compiled to a temporary
library; the pin checks below must reject every one of them."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import vsht_inputs as vi
from test_oracle_pins import EXTENDED_CASES, brute_vsh, lambda_explicit, point_at, scipy_Y

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "vsht_oracle.c")

MUTANTS = {
    "no_condon_shortley": ("            pmm = -pmm * sx * sqrtl", "            pmm = pmm * sx * sqrtl"),
    "negative_order_no_sign": ("        p = -p; /* Y_{l,-|m|}", "        p = p; /* Y_{l,-|m|}"),
    "cg_sign_C4": ("B0 += dl * -sqrt(", "B0 += dl * sqrt("),
    "cg_index_C1": ("sqrt((L + M) * (L + M - 1.0) / ((2.0 * L)", "sqrt((L + M) * (L + M + 1.0) / ((2.0 * L)"),
    "c_d_swapped": ("const double cl = sqrt((L + 1.0) / (2.0 * L + 1.0));",
                    "const double cl = sqrt(L / (2.0 * L + 1.0));"),
    "curl_sign": ("ycurl[2] = D0;", "ycurl[2] = -D0;"),
    "vsh2_transposed": ("ydiv[0] = -(Bp - Bm) / r2;", "ydiv[0] = -(Bp + Bm) / r2;"),
    "forward_no_conj": ("sa += conj(yd[c]) * Tk[c];", "sa += yd[c] * Tk[c];"),
    "forward_no_weight": ("pa[j] += w[k] * sa;", "pa[j] += sa;"),
    "adjoint_dropped_b": ("acc[c] += a[j] * yd[c] + b[j] * yc[c];", "acc[c] += a[j] * yd[c];"),
    "recurrence_B": ("return A * (z * p1 - B * p2);", "return A * (z * p1 + B * p2);"),
    "binary64_recurrence": ("typedef long double xreal;", "typedef double xreal;"),
}


def build_mutant(name, tmpdir):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, name
    path = os.path.join(tmpdir, name + ".c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = os.path.join(tmpdir, name + ".so")
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", so, path, "-lm"])
    lib = ctypes.CDLL(so)
    i64, i32, dp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    lib.vo_sph_harm.argtypes = [i32, i64, dp, dp]
    lib.vo_vsh.argtypes = [i32, i64, dp, dp, dp]
    lib.vo_forward.argtypes = [i32, i64, dp, dp, dp, dp, dp]
    lib.vo_adjoint.argtypes = [i32, dp, dp, i64, dp, dp]
    return lib


def p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def pins_pass(lib):
    """The quick pins; True only if all of them hold."""
    L = 4
    xyz, _ = vi.uniform_points(24, 41)
    n = len(xyz)
    Y = np.zeros((n, (L + 1) ** 2), np.complex128)
    lib.vo_sph_harm(L, n, p(xyz), p(Y))
    for l in range(L + 1):
        for m in range(-l, l + 1):
            if np.max(np.abs(Y[:, l * l + l + m] - scipy_Y(l, m, xyz))) > 1e-12:
                return False
    K = L * (L + 2)
    d = np.zeros((n, K, 3), np.complex128)
    c = np.zeros((n, K, 3), np.complex128)
    lib.vo_vsh(L, n, p(xyz), p(d), p(c))
    bd, bc = brute_vsh(L, xyz)
    if np.max(np.abs(d - bd)) > 1e-12 or np.max(np.abs(c - bc)) > 1e-12:
        return False
    gx, gw = vi.gl_grid(L)
    a, b = vi.random_coeffs(L, 0)
    T = np.zeros((len(gw), 3), np.complex128)
    lib.vo_adjoint(L, p(a), p(b), len(gw), p(gx), p(T))
    a2 = np.zeros(K, np.complex128)
    b2 = np.zeros(K, np.complex128)
    lib.vo_forward(L, len(gw), p(gx), p(gw), p(T), p(a2), p(b2))
    err = np.linalg.norm(np.concatenate([a2 - a, b2 - b])) / np.linalg.norm(np.concatenate([a, b]))
    if err >= 1e-12:
        return False
    # one extended-range value (seed below binary64's range, value of order one)
    theta, l, m = EXTENDED_CASES[0]
    z, xyz = point_at(theta)
    sign, lg = explicit_value(theta, l, m)
    Yb = np.zeros((1, (l + 1) ** 2), np.complex128)
    lib.vo_sph_harm(l, 1, p(xyz), p(Yb))
    ref = sign * 10.0 ** lg
    return abs(Yb[0, l * l + l + m].real - ref) <= 1e-10 * abs(ref)


_explicit = {}


def explicit_value(theta, l, m):
    if (theta, l, m) not in _explicit:
        _explicit[(theta, l, m)] = lambda_explicit(l, m, point_at(theta)[0])
    return _explicit[(theta, l, m)]


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_rejected(name):
    with tempfile.TemporaryDirectory() as td:
        lib = build_mutant(name, td)
        assert not pins_pass(lib), "planted mistake %s was not caught" % name


def test_unmutated_passes():
    with tempfile.TemporaryDirectory() as td:
        src = open(SRC).read()
        path = os.path.join(td, "orig.c")
        open(path, "w").write(src)
        MUTANTS["_identity"] = ("typedef double complex cplx;", "typedef double complex cplx;")
        try:
            lib = build_mutant("_identity", td)
        finally:
            del MUTANTS["_identity"]
        assert pins_pass(lib)
