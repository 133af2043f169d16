"""Batches of fields with uneven bandlimits: every stage as one launch over all
fields, replayed from a HIP graph.  The batched kernels run the same bodies as
the single-field kernels, so each field must equal its single-plan result
exactly, for every launch shape; the FP64 batch is also checked against the
oracle.  Graph replays are repeated with host synchronisation between them and
each replay is checked."""
import numpy as np
import pytest

import vsht_inputs as vi

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-11


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


def dev(torch, x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype=dtype, device="cuda")


def make_batch(torch, vsht, Ls, precision, seed0=100):
    grids = [vi.gl_grid(L) for L in Ls]
    bp = vsht.BatchPlan(Ls, grids, precision=precision)
    coeffs = [vi.random_coeffs(L, seed0 + i) for i, L in enumerate(Ls)]
    a = [dev(torch, c[0], bp.dtype) for c in coeffs]
    b = [dev(torch, c[1], bp.dtype) for c in coeffs]
    return bp, grids, coeffs, a, b


def single_results(torch, vsht, Ls, grids, a, b, precision):
    out = []
    for L, (xyz, w), ai, bi in zip(Ls, grids, a, b):
        p = vsht.Plan(L, xyz, w, precision=precision)
        T = p.adjoint(ai, bi)
        a2, b2 = p.forward(T)
        torch.cuda.synchronize()
        out.append((T.cpu().numpy(), a2.cpu().numpy(), b2.cpu().numpy()))
        p.close()
    return out


LS_MIXED = [1, 7, 16, 33, 64, 100, 129, 40]   # 1..3 tiles of 64 ring pairs, odd and even ring counts


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "bf16x6"])
def test_batch_equals_single_plans(torch, vsht, precision):
    print("[case] batch vs single plans", precision, LS_MIXED, flush=True)
    bp, grids, coeffs, a, b = make_batch(torch, vsht, LS_MIXED, precision)
    ref = single_results(torch, vsht, LS_MIXED, grids, a, b, precision)
    for cfg in [dict(adj_nw=4, fwd_merge=0, lpt=1, ring_nt=256, chains=0),
                dict(adj_nw=1, fwd_merge=1, lpt=0, ring_nt=512, chains=0),
                dict(adj_nw=2, fwd_merge=1, lpt=1, ring_nt=256, chains=0)]:
        bp.set_config(**cfg)
        assert bp.config() == cfg
        T, a2, b2 = bp.roundtrip(a, b)
        torch.cuda.synchronize()
        for f in range(len(LS_MIXED)):
            assert np.array_equal(T[f].cpu().numpy(), ref[f][0]), (cfg, f)
            assert np.array_equal(a2[f].cpu().numpy(), ref[f][1]), (cfg, f)
            assert np.array_equal(b2[f].cpu().numpy(), ref[f][2]), (cfg, f)
    bp.close()


@pytest.mark.skip(reason="parallel size-class chains are switched off in the library: one run crashed "
                         "(segmentation fault in the host process) during an autotune that captured and "
                         "replayed the multi-branch graphs, and the cause is not found")
def test_batch_chains_equal_single_plans(torch, vsht):
    """Size-class chains (three parallel branches of the captured graph) give the
    single plans' results bit for bit."""
    print("[case] batch chains vs single plans fp32", LS_MIXED, flush=True)
    bp, grids, coeffs, a, b = make_batch(torch, vsht, LS_MIXED, "fp32")
    ref = single_results(torch, vsht, LS_MIXED, grids, a, b, "fp32")
    bp.set_config(adj_nw=4, fwd_merge=1, lpt=0, ring_nt=512, chains=1)
    T, a2, b2 = bp.roundtrip(a, b)
    torch.cuda.synchronize()
    for f in range(len(LS_MIXED)):
        assert np.array_equal(T[f].cpu().numpy(), ref[f][0]), f
        assert np.array_equal(a2[f].cpu().numpy(), ref[f][1]), f
    bp.close()


def test_batch_fp64_vs_oracle_and_replays(torch, vsht, orc):
    Ls = [3, 16, 24, 65]
    print("[case] batch fp64 vs oracle, replays", Ls, flush=True)
    bp, grids, coeffs, a, b = make_batch(torch, vsht, Ls, "fp64")
    T_ref = [orc.adjoint(L, c[0], c[1], g[0]) for L, c, g in zip(Ls, coeffs, grids)]
    T = bp.empty_fields()
    a2 = bp.empty_coeffs()
    b2 = bp.empty_coeffs()
    for rep in range(4):
        for t in T:
            t.zero_()
        torch.cuda.synchronize()
        bp.roundtrip(a, b, T, a2, b2)
        torch.cuda.synchronize()
        for f, L in enumerate(Ls):
            assert rel_l2(T[f].cpu().numpy(), T_ref[f]) < FP64_TOL, (rep, f)
            c = np.concatenate([a2[f].cpu().numpy(), b2[f].cpu().numpy()])
            assert rel_l2(c, np.concatenate(coeffs[f])) < FP64_TOL, (rep, f)
    # separate directions, and new buffers (rebinding)
    T2 = bp.adjoint(a, b)
    a3, b3 = bp.forward(T2)
    torch.cuda.synchronize()
    for f in range(len(Ls)):
        assert np.array_equal(T2[f].cpu().numpy(), T[f].cpu().numpy())
        assert np.array_equal(a3[f].cpu().numpy(), a2[f].cpu().numpy())
    bp.close()


def test_batch_autotune_and_field_times(torch, vsht):
    Ls = [34, 48, 101, 259, 278, 395]
    print("[case] batch autotune fp32", Ls, flush=True)
    bp, grids, coeffs, a, b = make_batch(torch, vsht, Ls, "fp32")
    T, a2, b2 = bp.roundtrip(a, b)
    torch.cuda.synchronize()
    first = [x.cpu().numpy().copy() for x in a2]
    ms = bp.autotune(a, b, T, a2, b2, reps=2)
    assert ms > 0
    cfg = bp.config()
    assert cfg["adj_nw"] in (1, 2, 4) and cfg["chains"] == 0
    with pytest.raises(RuntimeError, match="EUNSUPPORTED"):
        bp.set_config(chains=1)  # parallel chains are switched off
    bp.roundtrip(a, b, T, a2, b2)
    t0, t1 = bp.field_times()
    torch.cuda.synchronize()
    for f in range(len(Ls)):
        assert np.array_equal(a2[f].cpu().numpy(), first[f])
    assert t0.shape == (len(Ls),) and np.all(t1 > t0) and np.min(t0) == 0.0
    print("[batch] autotuned", cfg, "%.3f ms" % ms, "latency us", np.round(t1 - t0, 1), flush=True)
    bp.close()


def test_batch_tune_cache(torch, vsht, tmp_path):
    """vsht_opts.tune_cache: the first autotune times the shapes and stores the
    fastest; a batch of the same field shapes reads it back without timing and
    takes the same shape; other shapes get their own entry."""
    print("[case] batch tune cache", flush=True)
    cache = str(tmp_path / "tune.txt")
    Ls = [8, 12, 20]
    grids = [vi.gl_grid(L) for L in Ls]

    def tuned(Ls_, grids_):
        bp = vsht.BatchPlan(Ls_, grids_, precision="fp32", tune_cache=cache)
        coeffs = [vi.random_coeffs(L, 300 + i) for i, L in enumerate(Ls_)]
        a = [dev(torch, c[0], bp.dtype) for c in coeffs]
        b = [dev(torch, c[1], bp.dtype) for c in coeffs]
        T, a2, b2 = bp.empty_fields(), bp.empty_coeffs(), bp.empty_coeffs()
        ms = bp.autotune(a, b, T, a2, b2, reps=2)
        cfg = bp.config()
        bp.close()
        return ms, cfg

    ms1, cfg1 = tuned(Ls, grids)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("b2:") and lines[0].split()[0].count(":") == 4
    assert len(lines[0].split()) == 7
    ms2, cfg2 = tuned(Ls, grids)
    assert cfg2 == cfg1 and ms2 == pytest.approx(ms1, rel=1e-5)
    assert len(open(cache).read().splitlines()) == 1  # read, not timed again
    tuned(Ls[:2], grids[:2])
    assert len(open(cache).read().splitlines()) == 2
