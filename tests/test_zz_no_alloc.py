"""The allocation-free forward (vsht_forward_static, its buffers in the library's
static device array) against vsht_forward on the same plan: the same kernels in
the same order, so the outputs must agree bit for bit.  Several calls in a row,
each later one on a smaller plan than the one before (the array keeps the
previous call's contents), in binary64 and binary32, including a plan whose
analysis is split over several workgroups per order (partial triangles in the
array too); plans the array cannot hold and scattered plans are refused."""
import numpy as np
import pytest

import vsht_inputs as vi

pytestmark = pytest.mark.gpu


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


def many_pair_grid(L, n_pairs, n_phi):
    """Mirrored rings (z_S = -z_N exactly) at equispaced colatitudes: more than 1024
    pairs at small size; the weights need not be a quadrature rule here."""
    th = np.pi * (np.arange(n_pairs) + 0.5) / (2 * n_pairs + 1)
    zn = np.cos(th)
    z = np.concatenate([zn, -zn[::-1]])
    s = np.sqrt((1.0 - z) * (1.0 + z))
    ph = 2.0 * np.pi * np.arange(n_phi) / n_phi
    xyz = np.stack([np.outer(s, np.cos(ph)), np.outer(s, np.sin(ph)), np.outer(z, np.ones(n_phi))],
                   axis=-1).reshape(-1, 3)
    w = np.full(len(xyz), 4.0 * np.pi / len(xyz))
    return xyz, w


def run_both(torch, vsht, plan, T):
    a1, b1 = plan.forward(T)
    a2 = torch.empty_like(a1)
    b2 = torch.empty_like(b1)
    st = vsht.vsht_forward_static(plan._h, T.data_ptr(), a2.data_ptr(), b2.data_ptr(),
                                  torch.cuda.current_stream().cuda_stream)
    assert st == 0, vsht.load_library().vsht_last_error().decode()
    torch.cuda.synchronize()
    return a1, b1, a2, b2


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_forward_matches_forward(torch, vsht, precision):
    cases = [("gl", 64), ("gl", 24), ("split", 6)]
    for kind, L in cases:
        print("[case] static forward", precision, kind, L, flush=True)
        if kind == "gl":
            xyz, w = vi.gl_grid(L)
        else:
            xyz, w = many_pair_grid(L, 1040, 14)
        plan = vsht.Plan(L, xyz, w, precision=precision)
        if kind == "split":
            assert plan.info()["n_pairs"] == 1040  # 17 tiles: two workgroups per order
        T = torch.from_numpy(vi.random_field(len(w), 40 + L)).to("cuda", plan.dtype)
        a1, b1, a2, b2 = run_both(torch, vsht, plan, T)
        assert torch.equal(a1, a2) and torch.equal(b1, b2), (precision, kind, L)
        assert torch.isfinite(a1).all() and a1.abs().max() > 0
        plan.close()


def test_static_forward_refusals(torch, vsht):
    from paper_1908_00041_amd import _binding as B
    dev = "cuda"
    # a scattered plan
    xyz, _ = vi.uniform_points(200, 7)
    plan = vsht.Plan(8, xyz, np.full(200, 4 * np.pi / 200), precision="fp64")
    assert plan.kind == "scattered"
    T = torch.zeros((200, 3), dtype=torch.complex128, device=dev)
    a = torch.zeros(80, dtype=torch.complex128, device=dev)
    st = vsht.vsht_forward_static(plan._h, T.data_ptr(), a.data_ptr(), a.data_ptr(), 0)
    assert st == B.VSHT_EUNSUPPORTED
    plan.close()
    # a plan without weights
    xyz, w = vi.gl_grid(8)
    plan = vsht.Plan(8, xyz, None, precision="fp64")
    T = torch.zeros((len(w), 3), dtype=torch.complex128, device=dev)
    st = vsht.vsht_forward_static(plan._h, T.data_ptr(), a.data_ptr(), a.data_ptr(), 0)
    assert st == B.VSHT_ENOWEIGHTS
    plan.close()
    # a plan larger than the array: FP64 GL at L = 1200 needs ~139 MB
    L = 1200
    xyz, w = vi.gl_grid(L)
    plan = vsht.Plan(L, xyz, w, precision="fp64")
    T = torch.zeros((len(w), 3), dtype=torch.complex128, device=dev)
    ab = torch.zeros(L * (L + 2), dtype=torch.complex128, device=dev)
    st = vsht.vsht_forward_static(plan._h, T.data_ptr(), ab.data_ptr(), ab.data_ptr(), 0)
    assert st == B.VSHT_EUNSUPPORTED
    assert b"static array" in vsht.load_library().vsht_last_error()
    plan.close()
