"""GPU parity of the scalar transforms (vsht_sht_forward / vsht_sht_adjoint)
against the oracle's orthonormal harmonics Y_{l,m} (Section 3) written out as
dense sums: f_{l,m} = sum_k w_k f_k conj(Y_{l,m}(x_k)) (Section 4.1) and
f(x_k) = sum_{l,m} f_{l,m} Y_{l,m}(x_k) (Section 4.2)."""
import numpy as np
import pytest

import vsht_inputs as vi

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11
# the mixed-precision bar of the vector transforms (relative L2 <= 1e-6)
FP32_TOL = 1e-6
# split-bf16 contractions: the bounds argued for the vector transforms (three
# products drop terms up to 3 * 2^-18 relative per product; six stay below binary32)
BF16X3_TOL = 3 * 2.0 ** -18
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


def random_scalar(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def grid(kind, L):
    return vi.gl_grid(L) if kind == "gl" else vi.reduced_gl_grid(L)


@pytest.mark.parametrize("kind,L,precision,tol", [
    ("gl", 1, "fp64", FP64_TOL), ("gl", 7, "fp64", FP64_TOL), ("gl", 33, "fp64", FP64_TOL),
    ("reduced", 40, "fp64", FP64_TOL), ("gl", 33, "fp32", FP32_TOL),
    ("reduced", 40, "fp32", FP32_TOL), ("gl", 33, "bf16x3", BF16X3_TOL),
    ("reduced", 40, "bf16x3", BF16X3_TOL), ("gl", 33, "bf16x6", BF16X6_TOL)])
def test_sht_forward_adjoint(torch, vsht, orc, kind, L, precision, tol):
    print("[case] sht", kind, L, precision, flush=True)
    xyz, w = grid(kind, L)
    Y = orc.sph_harm(L, xyz)                           # (n, (L+1)^2)
    plan = vsht.Plan(L, xyz, w, precision=precision)
    assert plan.kind == "rings"
    nc = vsht.vsht_num_sht_coeffs(L)
    assert nc == (L + 1) ** 2 == Y.shape[1]

    flm = random_scalar(nc, 21)
    f = plan.sht_adjoint(torch.from_numpy(flm).to(plan.dtype).cuda())
    torch.cuda.synchronize()
    e_adj = rel_l2(f.cpu().numpy(), Y @ flm)

    fr = random_scalar(len(w), 22)
    g = plan.sht_forward(torch.from_numpy(fr).to(plan.dtype).cuda())
    torch.cuda.synchronize()
    e_fwd = rel_l2(g.cpu().numpy(), Y.conj().T @ (w * fr))
    print("sht %s L=%d %s adjoint %.3e forward %.3e" % (kind, L, precision, e_adj, e_fwd))
    assert e_adj < tol and e_fwd < tol


def test_sht_roundtrip_gl(torch, vsht):
    """On a Gauss-Legendre grid with 2L+2 longitudes the quadrature is exact for
    products of two degree-L harmonics, so forward(adjoint(flm)) = flm."""
    L = 64
    xyz, w = vi.gl_grid(L)
    plan = vsht.Plan(L, xyz, w, precision="fp64")
    flm = random_scalar(vsht.vsht_num_sht_coeffs(L), 23)
    d = torch.from_numpy(flm).cuda()
    back = plan.sht_forward(plan.sht_adjoint(d))
    torch.cuda.synchronize()
    assert rel_l2(back.cpu().numpy(), flm) < FP64_TOL


def test_sht_errors(torch, vsht):
    L = 8
    xyz, w = vi.gl_grid(L)
    noweights = vsht.Plan(L, xyz, None, precision="fp64")
    f = torch.zeros(len(w), dtype=torch.complex128, device="cuda")
    with pytest.raises(vsht.VshtError):
        noweights.sht_forward(f)
    scattered = vsht.Plan(L, vi.uniform_points(50, 4)[0], None, precision="fp64")
    assert scattered.kind == "scattered"
    flm = torch.zeros(vsht.vsht_num_sht_coeffs(L), dtype=torch.complex128, device="cuda")
    with pytest.raises(vsht.VshtError):
        scattered.sht_adjoint(flm)
