"""GPU parity: the HIP path (through the C interface) against the CPU oracle
on the same seeded inputs.  FP64 bar: relative L2 <= 1e-11 over every
compared output; FP32 errors are asserted against a bound for a
single-precision contraction with binary64 Legendre values, and printed."""
import functools
import math

import numpy as np
import pytest

import vsht_inputs as vi

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11
# The mixed-precision path's stated bar: relative L2 <= 1e-6 against binary64
# (binary32 contraction with binary64 Legendre values, two-level binary32 sums,
# the ring pairs next to the poles in binary64).
FP32_TOL = 1e-6
# BF16x3: each operand x = hi + lo + r with |lo| <= 2^-9 |x| and |r| <= 2^-18 |x|;
# the dropped terms of one product (lo lo', r y, x r') are at most 3 * 2^-18
# = 1.14e-5 relative.  A transform's relative L2 error is bounded by that
# per-product bound (independent errors over terms of comparable size), and a
# round trip passes through two contractions.
BF16X3_TOL = 3 * 2.0 ** -18
BF16X3_RT_TOL = 2 * BF16X3_TOL
# BF16x6: three parts, |r| <= 2^-27 |x|; the dropped products (p1 p2', p2 p1',
# p2 p2' and the residuals) are below binary32's own rounding, so the binary32 bar holds.
BF16X6_TOL = FP32_TOL


def rel_l2(x, y):
    x = np.asarray(x).ravel()
    y = np.asarray(y).ravel()
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def vsht():
    import paper_1908_00041_amd as v
    v.load_library()
    return v


def to_dev(torch, x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype=dtype, device="cuda")


def run_adjoint(torch, plan, a, b):
    T = plan.adjoint(to_dev(torch, a, plan.dtype), to_dev(torch, b, plan.dtype))
    torch.cuda.synchronize()
    return T.cpu().numpy().astype(np.complex128)


def run_forward(torch, plan, T, weighted=True):
    a, b = plan.forward(to_dev(torch, T, plan.dtype), weighted=weighted)
    torch.cuda.synchronize()
    return a.cpu().numpy().astype(np.complex128), b.cpu().numpy().astype(np.complex128)


def print_case(*args):
    print("[case]", *args, flush=True)


# ---------------------------------------------------------------------------
# full parity on small and medium Gauss-Legendre grids
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [1, 2, 3, 16, 33, 64])
def test_gl_adjoint_forward_fp64(torch, vsht, orc, L):
    print_case("gl fp64", L)
    xyz, w = vi.gl_grid(L)
    a, b = vi.random_coeffs(L, 0)
    plan = vsht.Plan(L, xyz, w, precision="fp64")
    assert plan.kind == "rings"
    T_ref = orc.adjoint(L, a, b, xyz)
    T = run_adjoint(torch, plan, a, b)
    assert rel_l2(T, T_ref) < FP64_TOL
    # forward of a random (non-tangent) field, and of the band-limited one
    Tr = vi.random_field(len(w), 1)
    a_ref, b_ref = orc.forward(L, xyz, w, Tr)
    ga, gb = run_forward(torch, plan, Tr)
    assert rel_l2(np.concatenate([ga, gb]), np.concatenate([a_ref, b_ref])) < FP64_TOL
    ga, gb = run_forward(torch, plan, T_ref)
    assert rel_l2(np.concatenate([ga, gb]), np.concatenate([a, b])) < FP64_TOL


def test_gl_unweighted_forward_fp64(torch, vsht, orc):
    L = 20
    xyz, w = vi.gl_grid(L)
    plan = vsht.Plan(L, xyz, None, precision="fp64")
    Tr = vi.random_field(len(xyz), 2)
    a_ref, b_ref = orc.forward(L, xyz, np.ones(len(xyz)), Tr)
    ga, gb = run_forward(torch, plan, Tr, weighted=False)
    assert rel_l2(np.concatenate([ga, gb]), np.concatenate([a_ref, b_ref])) < FP64_TOL


@pytest.mark.parametrize("grid", ["odd_rings", "phase_shift", "alias", "nonuniform_w", "unpaired"])
def test_ring_grid_variants_fp64(torch, vsht, orc, grid):
    """Ring grids beyond GL: no equator ring, shifted longitudes, rings shorter
    than 2L+1 (bins alias), per-point weights, rings without a mirror."""
    print_case("variant", grid)
    L = 12
    rng = np.random.default_rng(5)
    if grid == "odd_rings":
        xyz, w = vi.gl_grid(L, n_theta=L + 2, n_phi=2 * L + 3)
    elif grid == "alias":
        xyz, w = vi.gl_grid(L, n_theta=L + 1, n_phi=L + 3)
    else:
        xyz, w = vi.gl_grid(L, n_theta=L + 1, n_phi=2 * L + 2)
    if grid == "phase_shift":
        nphi = 2 * L + 2
        ph = 2 * np.pi * np.arange(nphi) / nphi + 0.3
        z = xyz[::nphi, 2]
        s = np.sqrt((1 - z) * (1 + z))
        xyz = np.stack([np.outer(s, np.cos(ph)), np.outer(s, np.sin(ph)),
                        np.outer(z, np.ones(nphi))], axis=-1).reshape(-1, 3)
    if grid == "nonuniform_w":
        w = w * (1.0 + 0.1 * rng.standard_normal(len(w)))
    if grid == "unpaired":
        nphi = 2 * L + 2
        keep = np.ones(len(w), bool)
        keep[:2 * nphi] = False  # drop the two northernmost rings
        xyz, w = xyz[keep], w[keep]
    plan = vsht.Plan(L, xyz, w, precision="fp64")
    assert plan.kind == "rings"
    a, b = vi.random_coeffs(L, 7)
    T = run_adjoint(torch, plan, a, b)
    assert rel_l2(T, orc.adjoint(L, a, b, xyz)) < FP64_TOL
    Tr = vi.random_field(len(w), 8)
    ga, gb = run_forward(torch, plan, Tr)
    a_ref, b_ref = orc.forward(L, xyz, w, Tr)
    assert rel_l2(np.concatenate([ga, gb]), np.concatenate([a_ref, b_ref])) < FP64_TOL


@pytest.mark.parametrize("L,precision,tol", [(12, "fp64", FP64_TOL), (40, "fp64", FP64_TOL),
                                             (40, "fp32", FP32_TOL)])
def test_reduced_ring_grid(torch, vsht, orc, L, precision, tol):
    """Rings of unequal length (shorter than 2L+1 near the poles, so Fourier bins
    alias) and alternating phase: the ring path against the oracle's direct sums."""
    print_case("reduced rings", L, precision)
    xyz, w = vi.reduced_gl_grid(L)
    plan = vsht.Plan(L, xyz, w, precision=precision)
    assert plan.kind == "rings"
    a, b = vi.random_coeffs(L, 11)
    T = run_adjoint(torch, plan, a, b)
    e_adj = rel_l2(T, orc.adjoint(L, a, b, xyz))
    Tr = vi.random_field(len(w), 12)
    ga, gb = run_forward(torch, plan, Tr)
    a_ref, b_ref = orc.forward(L, xyz, w, Tr)
    e_fwd = rel_l2(np.concatenate([ga, gb]), np.concatenate([a_ref, b_ref]))
    print("reduced rings L=%d %s adjoint %.3e forward %.3e" % (L, precision, e_adj, e_fwd))
    assert e_adj < tol and e_fwd < tol


# HEALPix layout (equal-area rings of 4i points in the caps and 4 N_side in the
# belt, alternate belt rings shifted by half a step; the layout Section 6 names
# for future work): the ring path against the oracle's direct sums.  The
# forward is the weighted sum of eq. (fwdvsht2) with HEALPix's equal weights.
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_healpix_rings(torch, vsht, orc, precision, tol):
    nside, L = 16, 32
    print_case("healpix", nside, L, precision)
    xyz, w = vi.healpix_grid(nside)
    assert len(w) == 12 * nside * nside
    plan = vsht.Plan(L, xyz, w, precision=precision)
    assert plan.kind == "rings"
    a, b = vi.random_coeffs(L, 13)
    T = run_adjoint(torch, plan, a, b)
    e_adj = rel_l2(T, orc.adjoint(L, a, b, xyz))
    Tr = vi.random_field(len(w), 14)
    ga, gb = run_forward(torch, plan, Tr)
    a_ref, b_ref = orc.forward(L, xyz, w, Tr)
    e_fwd = rel_l2(np.concatenate([ga, gb]), np.concatenate([a_ref, b_ref]))
    print("healpix nside=%d L=%d %s adjoint %.3e forward %.3e" % (nside, L, precision, e_adj, e_fwd))
    assert e_adj < tol and e_fwd < tol
    plan.close()


# The double-Fourier-sphere path at L = 1024 (grid 4500 x 4500, the smallest
# 5-smooth length of at least 2(2L+1) whose DFT fits the LDS kernels) on 200,000
# uniform points plus both poles, equal weights: adjoint sampled at 64 points and
# forward (eq. (fwdvsht2)) sampled at 32 coefficients against the oracle.
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_scattered_grid_L1024(torch, vsht, orc, precision, tol):
    L = 1024
    print_case("scattered grid", L, precision)
    xyz, w = vi.uniform_points(200000, 91)
    xyz = np.concatenate([xyz, [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]])
    w = np.full(len(xyz), 4 * np.pi / len(xyz))
    plan = vsht.Plan(L, xyz, w, precision=precision)
    assert plan.kind == "scattered" and plan.info()["nfft_grid"] > 0
    a, b = vi.random_coeffs(L, 92)
    if precision != "fp64":
        a, b = (x.astype(np.complex64).astype(np.complex128) for x in (a, b))
    T = run_adjoint(torch, plan, a, b)
    pidx = np.concatenate([vi.sample_indices(len(w) - 2, 62, 93), [len(w) - 2, len(w) - 1]])
    e_adj = rel_l2(T[pidx], orc.adjoint(L, a, b, xyz[pidx]))
    Tr = vi.random_field(len(w), 94)
    if precision != "fp64":
        Tr = Tr.astype(np.complex64).astype(np.complex128)
    ga, gb = run_forward(torch, plan, Tr)
    cidx = vi.sample_indices(L * (L + 2), 32, 95)
    sa, sb = orc.forward_subset(L, xyz, w, Tr, cidx)
    e_fwd = rel_l2(np.concatenate([ga[cidx], gb[cidx]]), np.concatenate([sa, sb]))
    print("scattered grid L=%d %s grid %d adjoint %.3e forward %.3e"
          % (L, precision, plan.info()["nfft_grid"], e_adj, e_fwd), flush=True)
    assert e_adj < tol and e_fwd < tol
    plan.close()


def test_scattered_adjoint_fp64(torch, vsht, orc):
    L = 24
    xyz, _ = vi.uniform_points(700, 2)
    xyz = np.concatenate([xyz, [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]])
    plan = vsht.Plan(L, xyz, None, precision="fp64")
    assert plan.kind == "scattered"
    a, b = vi.random_coeffs(L, 3, scale="inv_sqrt_ll1")
    T = run_adjoint(torch, plan, a, b)
    T_ref = orc.adjoint(L, a, b, xyz)
    assert rel_l2(T, T_ref) < FP64_TOL
    assert rel_l2(T[-2:], T_ref[-2:]) < FP64_TOL  # the two poles


@pytest.mark.parametrize("L", [16, 64])
def test_gl_fp32(torch, vsht, orc, L):
    xyz, w = vi.gl_grid(L)
    a, b = vi.random_coeffs(L, 0)
    plan = vsht.Plan(L, xyz, w, precision="fp32")
    T_ref = orc.adjoint(L, a, b, xyz)
    T = run_adjoint(torch, plan, a, b)
    e_adj = rel_l2(T, T_ref)
    ga, gb = run_forward(torch, plan, T_ref)
    e_fwd = rel_l2(np.concatenate([ga, gb]), np.concatenate([a, b]))
    print("fp32 L=%d adjoint rel-L2 %.3e forward rel-L2 %.3e" % (L, e_adj, e_fwd))
    assert e_adj < FP32_TOL and e_fwd < FP32_TOL


@pytest.mark.parametrize("L,precision,tol", [(1, "bf16x3", BF16X3_TOL), (16, "bf16x3", BF16X3_TOL),
                                             (64, "bf16x3", BF16X3_TOL), (1, "bf16x6", BF16X6_TOL),
                                             (16, "bf16x6", BF16X6_TOL), (64, "bf16x6", BF16X6_TOL),
                                             (130, "bf16x6", BF16X6_TOL)])
def test_gl_bf16(torch, vsht, orc, L, precision, tol):
    print_case("gl", L, precision)
    xyz, w = vi.gl_grid(L)
    a, b = vi.random_coeffs(L, 0)
    plan = vsht.Plan(L, xyz, w, precision=precision)
    T_ref = orc.adjoint(L, a, b, xyz)
    T = run_adjoint(torch, plan, a, b)
    e_adj = rel_l2(T, T_ref)
    ga, gb = run_forward(torch, plan, T_ref)
    e_fwd = rel_l2(np.concatenate([ga, gb]), np.concatenate([a, b]))
    print("%s L=%d adjoint rel-L2 %.3e forward rel-L2 %.3e" % (precision, L, e_adj, e_fwd))
    assert e_adj < tol and e_fwd < tol


# ---------------------------------------------------------------------------
# L = 256 on the GL grid 257 x 514: sampled outputs
# ---------------------------------------------------------------------------
def test_gl_L256_sampled_fp64(torch, vsht, orc):
    L = 256
    print_case("gl fp64 sampled", L)
    xyz, w = vi.gl_grid(L)
    a, b = vi.random_coeffs(L, 0, scale="inv_sqrt_ll1")
    plan = vsht.Plan(L, xyz, w, precision="fp64")
    T = run_adjoint(torch, plan, a, b)
    pidx = vi.sample_indices(len(w), 96, 3)
    assert rel_l2(T[pidx], orc.adjoint(L, a, b, xyz[pidx])) < FP64_TOL
    cidx = vi.sample_indices(L * (L + 2), 96, 4)
    Tr = vi.random_field(len(w), 5)
    ga, gb = run_forward(torch, plan, Tr)
    sa, sb = orc.forward_subset(L, xyz, w, Tr, cidx)
    assert rel_l2(np.concatenate([ga[cidx], gb[cidx]]), np.concatenate([sa, sb])) < FP64_TOL
    # exact quadrature: forward(adjoint) recovers every coefficient
    ga, gb = run_forward(torch, plan, T)
    assert rel_l2(np.concatenate([ga, gb]), np.concatenate([a, b])) < FP64_TOL


# ---------------------------------------------------------------------------
# L = 1024 on the GL grid 1025 x 2050 in the launch configuration the
# benchmark times (one plan, adjoint then forward on the current stream).
# Inputs are binary32-representable, so every precision transforms the same
# values.  Checked: 4096 sampled points of the adjoint and 1024 sampled
# coefficients of the forward against the oracle; every output against the
# binary64 GPU path (itself held to the oracle at 1e-11 above); and the exact
# round trip Fwd(Adj(a, b)) = (a, b) at full size.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def l1024(torch, vsht, orc):
    L = 1024
    xyz, w = vi.gl_grid(L)
    a, b = vi.random_coeffs(L, 0)
    a = a.astype(np.complex64).astype(np.complex128)
    b = b.astype(np.complex64).astype(np.complex128)
    F = vi.random_field(len(w), 5).astype(np.complex64).astype(np.complex128)
    pidx = vi.sample_indices(len(w), 4096, 3)
    cidx = vi.sample_indices(L * (L + 2), 1024, 4)
    T_ref = orc.adjoint(L, a, b, xyz[pidx])
    fa_ref, fb_ref = orc.forward_subset(L, xyz, w, F, cidx)
    plan = vsht.Plan(L, xyz, w, precision="fp64")
    T64 = run_adjoint(torch, plan, a, b)
    ga, gb = run_forward(torch, plan, F)
    plan.close()
    return dict(L=L, xyz=xyz, w=w, a=a, b=b, F=F, pidx=pidx, cidx=cidx, T_ref=T_ref,
                f_ref=np.concatenate([fa_ref, fb_ref]), T64=T64, f64=np.concatenate([ga, gb]))


@pytest.mark.parametrize("precision,tol,rt_tol", [("fp64", FP64_TOL, FP64_TOL), ("fp32", FP32_TOL, FP32_TOL),
                                                  ("bf16x3", BF16X3_TOL, BF16X3_RT_TOL),
                                                  ("bf16x6", BF16X6_TOL, BF16X6_TOL)])
def test_gl_L1024(torch, vsht, l1024, precision, tol, rt_tol):
    d = l1024
    L = d["L"]
    print_case("gl L=1024", precision)
    plan = vsht.Plan(L, d["xyz"], d["w"], precision=precision)
    T = run_adjoint(torch, plan, d["a"], d["b"])
    e_adj = rel_l2(T[d["pidx"]], d["T_ref"])
    e_adj_full = rel_l2(T, d["T64"])
    ga, gb = run_forward(torch, plan, d["F"])
    g = np.concatenate([ga, gb])
    cidx, K = d["cidx"], L * (L + 2)
    e_fwd = rel_l2(np.concatenate([ga[cidx], gb[cidx]]), d["f_ref"])
    e_fwd_full = rel_l2(g, d["f64"])
    ra, rb = run_forward(torch, plan, T)
    e_rt = rel_l2(np.concatenate([ra, rb]), np.concatenate([d["a"], d["b"]]))
    plan.close()
    print("L=1024 %s adjoint %.3e (all points vs fp64 %.3e) forward %.3e (all vs fp64 %.3e) "
          "roundtrip %.3e" % (precision, e_adj, e_adj_full, e_fwd, e_fwd_full, e_rt))
    assert e_adj < tol and e_fwd < tol and e_rt < rt_tol
    if precision != "fp64":
        assert e_adj_full < tol and e_fwd_full < tol


# ---------------------------------------------------------------------------
# More than 1024 ring pairs: the analysis splits each order over several
# workgroups, whose partial triangles are added in a fixed order.  GL rule
# with 2101 rings (1050 pairs + the equator, 17 tiles of 64 pairs) of 82
# points at L = 40, every precision, against the oracle.
# ---------------------------------------------------------------------------
@functools.lru_cache(maxsize=None)
def many_ring_grid():
    return vi.gl_grid(40, n_theta=2101, n_phi=82)


@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL),
                                           ("bf16x3", BF16X3_TOL), ("bf16x6", BF16X6_TOL)])
def test_many_rings_split_analysis(torch, vsht, orc, precision, tol):
    L = 40
    print_case("2101 rings", L, precision)
    xyz, w = many_ring_grid()
    plan = vsht.Plan(L, xyz, w, precision=precision)
    assert plan.kind == "rings" and plan.info()["n_pairs"] == 1051
    Tr = vi.random_field(len(w), 13)
    a, b = vi.random_coeffs(L, 14)
    if precision != "fp64":
        Tr, a, b = (x.astype(np.complex64).astype(np.complex128) for x in (Tr, a, b))
    ga, gb = run_forward(torch, plan, Tr)
    a_ref, b_ref = orc.forward(L, xyz, w, Tr)
    e_fwd = rel_l2(np.concatenate([ga, gb]), np.concatenate([a_ref, b_ref]))
    T = run_adjoint(torch, plan, a, b)
    e_adj = rel_l2(T, orc.adjoint(L, a, b, xyz))
    print("2101 rings %s forward %.3e adjoint %.3e" % (precision, e_fwd, e_adj))
    assert e_fwd < tol and e_adj < tol


# ---------------------------------------------------------------------------
# The ring path has no atomics: two runs give bitwise equal outputs, on the
# GL grid at L = 256 and on the 2101-ring grid whose analysis is split.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_ring_path_bitwise_reproducible(torch, vsht, precision):
    print_case("reproducible", precision)
    for L in (256, 40):
        xyz, w = vi.gl_grid(L) if L == 256 else many_ring_grid()
        plan = vsht.Plan(L, xyz, w, precision=precision)
        a, b = vi.random_coeffs(L, 15)
        da, db = to_dev(torch, a, plan.dtype), to_dev(torch, b, plan.dtype)
        T1 = plan.adjoint(da, db).clone()
        T2 = plan.adjoint(da, db)
        a1, b1 = plan.forward(T1)
        a1, b1 = a1.clone(), b1.clone()
        a2, b2 = plan.forward(T1)
        torch.cuda.synchronize()
        assert torch.equal(T1, T2), (L, "adjoint")
        assert torch.equal(a1, a2) and torch.equal(b1, b2), (L, "forward")
        plan.close()


# ---------------------------------------------------------------------------
# The largest sizes served: GL grids with 2L+2 longitudes, the exact quadrature
# (round trip too), at L = 1535 (3072-point rings), at Table 3's L = 1750 (3502
# points, a radix-103 stage) and at L = 2047 (4096 points, the longest ring the
# ring kernels take); Table 3's largest bandlimit L = 2250 and the library's
# limit L = 4096, both on L+1 GL rings of 3072 points (the forward is checked as
# the discrete sum it is).  Above L ~ 1700 the seeds Lambda_{m,m} of functions that reach order one
# lie below binary64's range, so these cases run through start states computed
# with a carried exponent.  Sampled against the oracle.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L,nphi,nsample", [(1535, None, 32), (1750, None, 16), (2047, None, 16),
                                             (2250, 3072, 32), (4096, 3072, 16)])
def test_largest_sizes_sampled(torch, vsht, orc, L, nphi, nsample):
    print_case("largest sizes", L, nphi)
    xyz, w = vi.gl_grid(L, n_phi=nphi)
    plan = vsht.Plan(L, xyz, w, precision="fp64")
    assert plan.kind == "rings"
    a, b = vi.random_coeffs(L, 5)
    T = run_adjoint(torch, plan, a, b)
    pidx = vi.sample_indices(len(w), nsample, 6)
    e_adj = rel_l2(T[pidx], orc.adjoint(L, a, b, xyz[pidx]))
    cidx = vi.sample_indices(L * (L + 2), nsample, 7)
    ga, gb = run_forward(torch, plan, T)
    sa, sb = orc.forward_subset(L, xyz, w, T, cidx)
    e_fwd = rel_l2(np.concatenate([ga[cidx], gb[cidx]]), np.concatenate([sa, sb]))
    msg = "largest L=%d nphi=%d adjoint %.3e forward %.3e" % (L, len(w) // (L + 1), e_adj, e_fwd)
    if nphi is None:
        e_rt = rel_l2(np.concatenate([ga, gb]), np.concatenate([a, b]))
        msg += " roundtrip %.3e" % e_rt
        assert e_rt < FP64_TOL
    print(msg, flush=True)
    assert e_adj < FP64_TOL and e_fwd < FP64_TOL
    plan.close()


# ---------------------------------------------------------------------------
# Table 3's bandlimit on scattered points (the direct evaluation, L > 700): 48
# points at colatitudes where the seeds of order-one functions lie below
# binary64's range (theta = 0.3 to 0.6, where Lambda_{2250,m} ~ 1 for seeds
# near 1e-330), plus random points and both poles.
# ---------------------------------------------------------------------------
def test_scattered_direct_L2250(torch, vsht, orc):
    L = 2250
    print_case("scattered direct", L)
    rng = np.random.default_rng(61)
    th = np.concatenate([np.linspace(0.3, 0.6, 16), np.pi - np.linspace(0.3, 0.6, 8),
                         np.arccos(rng.uniform(-1, 1, 22))])
    ph = rng.uniform(0, 2 * np.pi, len(th))
    xyz = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    xyz /= np.linalg.norm(xyz, axis=1, keepdims=True)
    xyz = np.concatenate([xyz, [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]])
    plan = vsht.Plan(L, xyz, None, precision="fp64")
    assert plan.kind == "scattered"
    a, b = vi.random_coeffs(L, 62)
    T = run_adjoint(torch, plan, a, b)
    e = rel_l2(T, orc.adjoint(L, a, b, xyz))
    print("scattered direct L=%d adjoint %.3e" % (L, e), flush=True)
    assert e < FP64_TOL
    plan.close()


# ---------------------------------------------------------------------------
# Ring lengths with a prime factor beyond the generic radix: Bluestein DFT.
# GL grids at L = 66 (n_phi = 134 = 2 * 67) and L = 100 (202 = 2 * 101), a ring
# grid with prime n_phi = 131 (and a shifted longitude origin), and a mixed
# grid whose rings differ in length (generic and Bluestein in one plan).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["gl66", "gl100", "prime131", "mixed"])
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_bluestein_rings(torch, vsht, orc, case, precision, tol):
    print_case("bluestein", case, precision)
    if case == "gl66":
        L = 66
        xyz, w = vi.gl_grid(L)
    elif case == "gl100":
        L = 100
        xyz, w = vi.gl_grid(L)
    elif case == "prime131":
        L = 60
        nphi = 131
        z, wz = vi.gl_nodes(L + 1)
        ph = 2 * np.pi * np.arange(nphi) / nphi + 0.7
        s = np.sqrt((1 - z) * (1 + z))
        xyz = np.stack([np.outer(s, np.cos(ph)), np.outer(s, np.sin(ph)),
                        np.outer(z, np.ones(nphi))], axis=-1).reshape(-1, 3)
        w = np.repeat(wz * 2 * np.pi / nphi, nphi)
    else:
        L = 40
        z, wz = vi.gl_nodes(L + 1)
        lens = [82 if k % 2 == 0 else 89 for k in range(L + 1)]  # 89 is prime
        # mirror rings must have the same length for the grid to stay exact
        lens = [lens[min(k, L - k)] for k in range(L + 1)]
        pts, wts = [], []
        for k in range(L + 1):
            nphi = lens[k]
            ph = 2 * np.pi * np.arange(nphi) / nphi
            sk = np.sqrt((1 - z[k]) * (1 + z[k]))
            pts.append(np.stack([sk * np.cos(ph), sk * np.sin(ph), np.full(nphi, z[k])], axis=1))
            wts.append(np.full(nphi, wz[k] * 2 * np.pi / nphi))
        xyz, w = np.concatenate(pts), np.concatenate(wts)
    plan = vsht.Plan(L, xyz, w, precision=precision)
    assert plan.kind == "rings"
    a, b = vi.random_coeffs(L, 17)
    T = run_adjoint(torch, plan, a, b)
    e_adj = rel_l2(T, orc.adjoint(L, a, b, xyz))
    Tr = vi.random_field(len(w), 18)
    ga, gb = run_forward(torch, plan, Tr)
    a_ref, b_ref = orc.forward(L, xyz, w, Tr)
    e_fwd = rel_l2(np.concatenate([ga, gb]), np.concatenate([a_ref, b_ref]))
    print("bluestein %s %s adjoint %.3e forward %.3e" % (case, precision, e_adj, e_fwd))
    assert e_adj < tol and e_fwd < tol


# ---------------------------------------------------------------------------
# Scattered points through the double Fourier sphere (grid + window gather),
# against the oracle and against the direct evaluation.
# ---------------------------------------------------------------------------
def scattered_points(M, seed):
    xyz, w = vi.uniform_points(M, seed)
    poles = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    near = np.array([[1e-9, 0.0, np.sqrt(1 - 1e-18)], [0.0, -3e-7, -np.sqrt(1 - 9e-14)]])
    xyz = np.concatenate([xyz, poles, near])
    return xyz, np.full(len(xyz), 4 * np.pi / len(xyz))


@pytest.mark.parametrize("L,precision,tol", [(8, "fp64", FP64_TOL), (64, "fp64", FP64_TOL),
                                             (64, "fp32", FP32_TOL), (45, "bf16x3", BF16X3_TOL),
                                             (45, "bf16x6", BF16X6_TOL)])
def test_scattered_grid_vs_oracle(torch, vsht, orc, L, precision, tol):
    print_case("scattered grid", L, precision)
    xyz, w = scattered_points(1500, 21)
    plan = vsht.Plan(L, xyz, w, precision=precision)
    assert plan.kind == "scattered" and plan.info()["nfft_grid"] > 0
    a, b = vi.random_coeffs(L, 22)
    T = run_adjoint(torch, plan, a, b)
    T_ref = orc.adjoint(L, a, b, xyz)
    err = rel_l2(T, T_ref)
    err_poles = rel_l2(T[-4:], T_ref[-4:])
    print("scattered grid L=%d %s rel-L2 %.3e (poles %.3e)" % (L, precision, err, err_poles))
    assert err < tol and err_poles < 10 * tol


def test_scattered_grid_vs_direct(torch, vsht):
    L = 40
    print_case("scattered grid vs direct", L)
    xyz, w = scattered_points(3000, 23)
    a, b = vi.random_coeffs(L, 24)
    pg = vsht.Plan(L, xyz, w, precision="fp64")
    pd = vsht.Plan(L, xyz, w, precision="fp64", scattered="direct")
    assert pg.info()["nfft_grid"] > 0 and pd.info()["nfft_grid"] == 0
    # the direct evaluation divides the spin-frame sums by sin(theta), so it
    # loses digits within ~1e-6 of a pole (exact poles use the limit); compare
    # away from those two points
    keep = np.hypot(xyz[:, 0], xyz[:, 1]) > 1e-6
    keep |= np.hypot(xyz[:, 0], xyz[:, 1]) == 0
    Tg, Td = run_adjoint(torch, pg, a, b), run_adjoint(torch, pd, a, b)
    assert rel_l2(Tg[keep], Td[keep]) < FP64_TOL


def test_scattered_grid_L256_sampled(torch, vsht, orc):
    """M = 4 L^2 = 262,144 uniform points at L = 256 (plus both poles), sampled."""
    L = 256
    print_case("scattered grid L=256 M=262144")
    xyz, w = vi.uniform_points(4 * L * L, 2)
    xyz = np.concatenate([xyz, [[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]]])
    w = np.full(len(xyz), 4 * np.pi / len(xyz))
    a, b = vi.random_coeffs(L, 0, scale="inv_sqrt_ll1")
    plan = vsht.Plan(L, xyz, w, precision="fp64")
    T = run_adjoint(torch, plan, a, b)
    pidx = np.concatenate([vi.sample_indices(len(xyz) - 2, 64, 3), [len(xyz) - 2, len(xyz) - 1]])
    err = rel_l2(T[pidx], orc.adjoint(L, a, b, xyz[pidx]))
    print("scattered grid L=256 sampled rel-L2 %.3e" % err)
    assert err < FP64_TOL


@pytest.mark.parametrize("L,precision,tol", [(8, "fp64", FP64_TOL), (48, "fp64", FP64_TOL),
                                             (48, "fp32", FP32_TOL)])
def test_scattered_forward_vs_oracle(torch, vsht, orc, L, precision, tol):
    """Forward transform at scattered points (the transpose of the grid path)."""
    print_case("scattered forward", L, precision)
    xyz, w = scattered_points(1200, 31)
    w = w * (1.0 + 0.3 * np.random.default_rng(32).random(len(w)))
    plan = vsht.Plan(L, xyz, w, precision=precision)
    Tr = vi.random_field(len(w), 33)
    ga, gb = run_forward(torch, plan, Tr)
    a_ref, b_ref = orc.forward(L, xyz, w, Tr)
    e_w = rel_l2(np.concatenate([ga, gb]), np.concatenate([a_ref, b_ref]))
    ua, ub = run_forward(torch, plan, Tr, weighted=False)
    a1, b1 = orc.forward(L, xyz, np.ones(len(w)), Tr)
    e_u = rel_l2(np.concatenate([ua, ub]), np.concatenate([a1, b1]))
    print("scattered forward L=%d %s weighted %.3e unweighted %.3e" % (L, precision, e_w, e_u))
    assert e_w < tol and e_u < tol


def test_scattered_dot_product(torch, vsht):
    """<Adj(a, b), T> = <(a, b), Fwd_unweighted(T)> on the grid path (FP64)."""
    L = 30
    print_case("scattered dot test", L)
    xyz, w = scattered_points(2000, 41)
    plan = vsht.Plan(L, xyz, w)
    a, b = vi.random_coeffs(L, 42)
    T = vi.random_field(len(w), 43)
    lhs = np.vdot(T, run_adjoint(torch, plan, a, b))
    fa, fb = run_forward(torch, plan, T, weighted=False)
    rhs = np.vdot(np.concatenate([fa, fb]), np.concatenate([a, b]))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_scattered_direct_forward_unsupported(torch, vsht):
    from paper_1908_00041_amd import _binding as B
    xyz, w = scattered_points(100, 51)
    plan = vsht.Plan(8, xyz, w, scattered="direct")
    with pytest.raises(B.VshtError) as ei:
        run_forward(torch, plan, vi.random_field(len(w), 52))
    assert ei.value.status == B.VSHT_EUNSUPPORTED


# ---------------------------------------------------------------------------
# Buffers that do not start on a whole complex element are refused before any
# launch (single plans and the *_many calls).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_misaligned_buffers_rejected(torch, vsht, precision):
    print_case("misaligned buffers", precision)
    from paper_1908_00041_amd import _binding as B
    L = 8
    xyz, w = vi.gl_grid(L)
    plan = vsht.Plan(L, xyz, w, precision=precision)
    K = vi.num_coeffs(L)
    cdt = plan.dtype
    T = torch.zeros((len(w) + 1, 3), dtype=cdt, device="cuda")
    a = torch.zeros(K + 1, dtype=cdt, device="cuda")
    b = torch.zeros(K + 1, dtype=cdt, device="cuda")
    half = T.element_size() // 2  # half a complex element
    bad = T.data_ptr() + half
    assert B.vsht_forward(plan._h, bad, a.data_ptr(), b.data_ptr(), None) == B.VSHT_EINVAL
    assert "aligned" in B.load_library().vsht_last_error().decode()
    assert B.vsht_adjoint(plan._h, a.data_ptr(), b.data_ptr() + half, T.data_ptr(), None) == B.VSHT_EINVAL
    assert B.vsht_forward_many(plan._h, 1, T.data_ptr(), a.data_ptr() + half, b.data_ptr(), 0,
                               None) == B.VSHT_EINVAL
    # aligned buffers still work
    assert B.vsht_forward(plan._h, T.data_ptr(), a.data_ptr(), b.data_ptr(), None) == B.VSHT_OK
    torch.cuda.synchronize()
    plan.close()


# ---------------------------------------------------------------------------
# Plan options: VSHT_OPT_NO_FOLD (every ring its own pair) gives the oracle's
# values like the folded plan; nfft_eps sets the scattered grid path's accuracy.
# ---------------------------------------------------------------------------
def test_no_fold_option(torch, vsht, orc):
    L = 24
    print_case("no fold", L)
    xyz, w = vi.gl_grid(L)
    plan = vsht.Plan(L, xyz, w, precision="fp64", fold=False)
    info = plan.info()
    assert info["kind"] == 0 and info["n_pairs"] == info["n_rings"] == L + 1
    assert plan.workspace_bytes() > 0
    a, b = vi.random_coeffs(L, 71)
    T = run_adjoint(torch, plan, a, b)
    e_adj = rel_l2(T, orc.adjoint(L, a, b, xyz))
    Tr = vi.random_field(len(w), 72)
    ga, gb = run_forward(torch, plan, Tr)
    a_ref, b_ref = orc.forward(L, xyz, w, Tr)
    e_fwd = rel_l2(np.concatenate([ga, gb]), np.concatenate([a_ref, b_ref]))
    print("no fold L=%d adjoint %.3e forward %.3e" % (L, e_adj, e_fwd), flush=True)
    assert e_adj < FP64_TOL and e_fwd < FP64_TOL
    plan.close()


@pytest.mark.parametrize("eps", [1e-5, 1e-9])
def test_nfft_eps_option(torch, vsht, orc, eps):
    L = 32
    print_case("nfft_eps", eps)
    xyz, _ = vi.uniform_points(3000, 73)
    plan = vsht.Plan(L, xyz, None, precision="fp64", nfft_eps=eps)
    assert plan.kind == "scattered" and plan.info()["nfft_grid"] > 0
    a, b = vi.random_coeffs(L, 74)
    e = rel_l2(run_adjoint(torch, plan, a, b), orc.adjoint(L, a, b, xyz))
    print("nfft_eps %.0e adjoint %.3e" % (eps, e), flush=True)
    assert e <= 10 * eps            # the accuracy asked for
    assert e >= 1e-4 * eps          # and not the default's: the window did narrow
    plan.close()
