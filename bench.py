#!/usr/bin/env python3
"""Benchmark: forward + adjoint VSHT at L = 1024 on one MI355X.

Workload (one "step"): the adjoint transform of seeded random coefficients
(a, b) (re, im iid N(0,1), scaled by 1/l) onto the Gauss-Legendre grid of
1025 x 2050 = 2,101,250 points, then the forward transform of that field back
to coefficients.  Inputs are resident in HBM before the timed region.

Printed: ONE JSON line with the headline FP64 number (`value`, fwd+adj
transforms/s), the roofline record of the dominant kernel (HIP-event
durations measured here), the error against the CPU oracle on sampled outputs,
the oracle itself timed on the host (`cpu_baseline`), and the same
measurements for the lower-precision variants under `variants`.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--L 1024]
                    [--oracle-coeffs C] [--oracle-points P] [--no-oracle]
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_TFLOPS = 78.6   # dense MFMA peaks of the MI355X
FP32_MFMA_TFLOPS = 157.3
BF16_MFMA_TFLOPS = 2516.6
KERNEL_SRC = os.path.join(ROOT, "paper_1908_00041_amd", "csrc", "vsht_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def measured_traffic(kernel, prec, L):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None
    when there is none or the kernel source changed after it was measured."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        with open(KERNEL_SRC, "rb") as f:
            digest = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha256") != digest or rec.get("L") != L:
        return None
    table = rec.get("bytes_per_launch", {})
    if kernel in table:
        return int(table[kernel])
    # templated kernels: "<name><double>" or, for the ring stages, "<name><double, 512>"
    head = "%s<%s" % (kernel, "double" if prec == "fp64" else "float")
    hits = [v for k, v in table.items() if k == head + ">" or k.startswith(head + ",")]
    return int(hits[0]) if len(hits) == 1 else None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def folded_elements(L, n_pairs):
    """(m >= 0, m <= l' <= L+1, ring pair) elements of one Legendre stage as this
    library runs it (the spin-frame form, degrees up to L+1)."""
    return n_pairs * ((L + 2) * (L + 3) // 2 - 1)


def method_elements(L):
    """E(L) = ((L+1)(L+2)/2) ceil((L+1)/2): the folded (l, m >= 0, ring pair)
    elements of the method's own dense Legendre contraction on the GL grid with
    L+1 rings, 32 flops each per direction (two functions dP and mP/s, eight real
    columns, multiply-add)."""
    return (L + 1) * (L + 2) // 2 * ((L + 2) // 2)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def time_steps(torch, plan, a, b, steps, warmup):
    for _ in range(warmup):
        T = plan.adjoint(a, b)
        plan.forward(T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        T = plan.adjoint(a, b)
        a2, b2 = plan.forward(T)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, T, a2, b2


def stage_profile(torch, plan, a, b, reps):
    plan.set_stage_timing(True)
    plan.stage_times()
    for _ in range(reps):
        T = plan.adjoint(a, b)
        plan.forward(T)
    torch.cuda.synchronize()
    st = plan.stage_times()
    plan.set_stage_timing(False)
    return {k: (ms / c if c else 0.0) for k, (ms, c) in st.items() if c}


def run_l256(torch, vsht, vi, args):
    """L = 256: GL grid 257 x 514 forward+adjoint (FP64, FP32) and the adjoint at M = 4 L^2
    = 262,144 points uniform on the sphere with weights 4 pi / M (FP64, FP32), coefficients
    scaled 1/sqrt(l(l+1)); errors on sampled outputs against the oracle unless --no-oracle."""
    dev = torch.device("cuda", 0)
    L = 256
    a_np, b_np = vi.random_coeffs(L, 0, scale="inv_sqrt_ll1")
    xyz, w = vi.gl_grid(L)
    sx, _ = vi.uniform_points(4 * L * L, 2)
    sw = np.full(len(sx), 4 * np.pi / len(sx))
    pidx = vi.sample_indices(len(sx), 64, 3)
    ref = None
    if not args.no_oracle:
        import oracle
        oracle.build(force=False)
        ref = oracle.adjoint(L, a_np, b_np, sx[pidx])
    out = {}
    for prec in ("fp64", "fp32"):
        cdt = torch.complex128 if prec == "fp64" else torch.complex64
        a = torch.from_numpy(a_np).to(dev, cdt)
        b = torch.from_numpy(b_np).to(dev, cdt)
        plan = vsht.Plan(L, xyz, w, precision=prec)
        sec, T, a2, b2 = time_steps(torch, plan, a, b, args.steps, args.warmup)
        rt = rel_l2(np.concatenate([a2.cpu().numpy(), b2.cpu().numpy()]), np.concatenate([a_np, b_np]))
        plan.close()
        sp = vsht.Plan(L, sx, sw, precision=prec)
        for _ in range(args.warmup):
            Ts = sp.adjoint(a, b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Ts = sp.adjoint(a, b)
        torch.cuda.synchronize()
        ssec = (time.perf_counter() - t0) / args.steps
        r = {"gl_ms_per_fwd_adj": round(sec * 1e3, 4), "gl_roundtrip_rel_l2": rt,
             "scattered_points": len(sx), "scattered_ms_per_adjoint": round(ssec * 1e3, 4),
             "scattered_points_per_s": round(len(sx) / ssec, 1), "nfft_grid": sp.info()["nfft_grid"]}
        if ref is not None:
            r["scattered_adjoint_vs_oracle_rel_l2"] = rel_l2(Ts.cpu().numpy()[pidx].astype(np.complex128), ref)
        sp.close()
        out[prec] = r
        log("L=256 %s: GL fwd+adj %.3f ms, scattered adjoint %.3f ms" % (prec, sec * 1e3, ssec * 1e3))
    return out


def run_table3(torch, vsht, vi, args):
    """The bandlimits of the paper's timing table: FP64 forward+adjoint on the GL grid
    (L+1) x (2L+2) (N = 2(L+1)^2 points, M = L^2 + 2L coefficients), random coefficients
    scaled 1/l.  Bandlimits whose rings do not fit the ring DFT stages (L = 2000: 4002
    points per ring, L = 2250: 4502) run on the scattered path and are not timed."""
    dev = torch.device("cuda", 0)
    out = []
    for L in [int(x) for x in args.table3.split(",") if x]:
        xyz, w = vi.gl_grid(L)
        t0 = time.perf_counter()
        plan = vsht.Plan(L, xyz, w, precision="fp64")
        t_plan = time.perf_counter() - t0
        if plan.kind != "rings":
            log("table3: L=%d planned as %s, not timed" % (L, plan.kind))
            out.append({"L": L, "points": len(w), "plan": plan.kind})
            plan.close()
            continue
        a_np, b_np = vi.random_coeffs(L, 0)
        a = torch.from_numpy(a_np).to(dev)
        b = torch.from_numpy(b_np).to(dev)
        sec, T, a2, b2 = time_steps(torch, plan, a, b, max(3, args.steps // 4), 1)
        rt = rel_l2(np.concatenate([a2.cpu().numpy(), b2.cpu().numpy()]), np.concatenate([a_np, b_np]))
        plan.close()
        del T, a2, b2
        log("table3: L=%d, %d points: fwd+adj %.3f ms, round trip %.2e, plan %.2f s"
            % (L, len(w), sec * 1e3, rt, t_plan))
        out.append({"L": L, "points": len(w), "coefficients": L * (L + 2), "ms_per_fwd_adj": round(sec * 1e3, 4),
                    "roundtrip_rel_l2": rt, "plan_s": round(t_plan, 2)})
    return out


def run_batched(torch, vsht, vi, args):
    """Many fields of uneven bandlimit, each on its own GL grid (L+1) x (2L+2), complex64,
    coefficients scaled 1/l: adjoint then forward of every field, one graph replay."""
    dev = torch.device("cuda", 0)
    Ls = [int(L) for L in vi.batch_bandlimits(args.batch_fields, seed=1)]
    log("batch: %d fields, L in [%d, %d], mean %.1f" % (len(Ls), min(Ls), max(Ls), np.mean(Ls)))
    grids = [vi.gl_grid(L) for L in Ls]
    t0 = time.perf_counter()
    bp = vsht.BatchPlan(Ls, grids, precision="fp32")
    t_plan = time.perf_counter() - t0
    rng_seeds = [1000 + f for f in range(len(Ls))]
    coeffs = [vi.random_coeffs(L, sd) for L, sd in zip(Ls, rng_seeds)]
    a = [torch.from_numpy(c[0]).to(dev, torch.complex64) for c in coeffs]
    b = [torch.from_numpy(c[1]).to(dev, torch.complex64) for c in coeffs]
    T, a2, b2 = bp.empty_fields(), bp.empty_coeffs(), bp.empty_coeffs()
    tuned_ms = bp.autotune(a, b, T, a2, b2, reps=3)
    cfg = bp.config()
    log("batch: autotuned %s (%.3f ms)" % (cfg, tuned_ms))
    for _ in range(args.warmup):
        bp.roundtrip(a, b, T, a2, b2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bp.roundtrip(a, b, T, a2, b2)
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    s0, s1 = bp.field_times()
    lat = s1 - s0
    # errors of four fields against single-field FP64 plans on the GPU
    errs = []
    for f in sorted(set([0, int(np.argmax(Ls)), int(np.argmin(Ls)), len(Ls) // 2])):
        xyz, w = grids[f]
        p = vsht.Plan(Ls[f], xyz, w, precision="fp64")
        T64 = p.adjoint(torch.from_numpy(coeffs[f][0]).to(dev), torch.from_numpy(coeffs[f][1]).to(dev))
        torch.cuda.synchronize()
        errs.append(rel_l2(T[f].cpu().numpy().astype(np.complex128), T64.cpu().numpy()))
        errs.append(rel_l2(np.concatenate([a2[f].cpu().numpy(), b2[f].cpu().numpy()]).astype(np.complex128),
                           np.concatenate(coeffs[f])))
        p.close()
    bp.close()
    log("batch: %.3f ms per batch, %.0f fields/s, field latency p50 %.0f us, p99 %.0f us"
        % (sec * 1e3, len(Ls) / sec, np.percentile(lat, 50), np.percentile(lat, 99)))
    return {"fields": len(Ls), "L_min": min(Ls), "L_max": max(Ls), "L_mean": round(float(np.mean(Ls)), 1),
            "precision": "fp32", "ms_per_batch": round(sec * 1e3, 4),
            "fields_per_s": round(len(Ls) / sec, 1),
            "latency_us_p50": round(float(np.percentile(lat, 50)), 1),
            "latency_us_p99": round(float(np.percentile(lat, 99)), 1),
            "autotuned": cfg, "plan_s": round(t_plan, 2),
            "max_rel_l2_vs_fp64_single": max(errs),
            "note": "adjoint then forward of every field per replay; latency = first work item start to "
                    "last work item end of each field (device wall clock)"}


def run_differentiable(torch, vsht, vi, args):
    """Loss ||Adj(a, b) - T_target||^2 over a batch of fields at L=512 (GL 513 x 1026), FP32;
    one step = the transform and its backward (the unit-weight forward)."""
    dev = torch.device("cuda", 0)
    L, F = 512, args.grad_fields
    xyz, w = vi.gl_grid(L)
    plan = vsht.Plan(L, xyz, w, precision="fp32")
    K = L * (L + 2)
    at = np.stack([vi.random_coeffs(L, 4 + 100 * f)[0] for f in range(F)])
    bt = np.stack([vi.random_coeffs(L, 4 + 100 * f)[1] for f in range(F)])
    Tt = plan.adjoint_many(torch.from_numpy(at).to(dev, torch.complex64),
                           torch.from_numpy(bt).to(dev, torch.complex64))
    rng = np.random.default_rng(5)
    noise = 0.1 * (rng.standard_normal((F, len(w), 3)) + 1j * rng.standard_normal((F, len(w), 3)))
    Tt = Tt + torch.from_numpy(noise).to(dev, torch.complex64)
    a0 = np.stack([vi.random_coeffs(L, 31 + f)[0] for f in range(F)])
    b0 = np.stack([vi.random_coeffs(L, 31 + f)[1] for f in range(F)])
    a = torch.from_numpy(a0).to(dev, torch.complex64).requires_grad_()
    b = torch.from_numpy(b0).to(dev, torch.complex64).requires_grad_()

    def step():
        a.grad = None
        b.grad = None
        r = vsht.adjoint_vsht(plan, a, b) - Tt
        loss = torch.view_as_real(r).square().sum()  # sum of |r|^2 over points and fields
        loss.backward()
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    plan.close()
    # error of the FP32 gradient of field 0 against the same step on the FP64 path
    # (same binary32-representable inputs)
    p64 = vsht.Plan(L, xyz, w, precision="fp64")
    a64 = a.detach()[0].to(torch.complex128).requires_grad_()
    b64 = b.detach()[0].to(torch.complex128).requires_grad_()
    r64 = vsht.adjoint_vsht(p64, a64, b64) - Tt[0].to(torch.complex128)
    (r64.real ** 2 + r64.imag ** 2).sum().backward()
    g64 = torch.cat([a64.grad, b64.grad]).cpu().numpy()
    g32 = torch.cat([a.grad[0], b.grad[0]]).cpu().numpy().astype(np.complex128)
    p64.close()
    gerr = rel_l2(g32, g64)
    log("differentiable: %.3f ms per step (%d fields, L=%d), gradient error vs fp64 %.2e"
        % (sec * 1e3, F, L, gerr))
    return {"fields": F, "L": L, "precision": "fp32", "ms_per_step": round(sec * 1e3, 4),
            "fields_per_s": round(F / sec, 1), "grad_rel_l2_vs_fp64": gerr,
            "note": "loss = ||Adj(a,b) - T_target||^2 summed over fields; step = adjoint of every field, "
                    "loss, and backward through the unit-weight forward kernels"}


def rel_l2(x, y):
    x = np.asarray(x).ravel()
    y = np.asarray(y).ravel()
    return float(np.linalg.norm(x - y) / max(np.linalg.norm(y), 1e-300))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=1024)
    ap.add_argument("--oracle-coeffs", type=int, default=4096)
    ap.add_argument("--oracle-points", type=int, default=4096)
    ap.add_argument("--no-oracle", action="store_true")
    ap.add_argument("--precisions", default="fp64,fp32,bf16x3,bf16x6",
                    help='L=1024 precisions to time ("" runs only the other legs, without a result line)')
    ap.add_argument("--l256", type=int, default=1,
                    help="also time L=256: GL 257 x 514 forward+adjoint and the adjoint at 4 L^2 scattered points")
    ap.add_argument("--batch-fields", type=int, default=256,
                    help="batched workload: this many complex64 fields, L uniform in [32, 512] (0: skip)")
    ap.add_argument("--grad-fields", type=int, default=8,
                    help="differentiable workload: this many fields at L=512, FP32 (0: skip)")
    ap.add_argument("--table3", default="",
                    help="comma-separated bandlimits: FP64 forward+adjoint on their GL grids "
                         "(e.g. 250,500,750,1000,1250,1500,1750; empty: skip)")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the transform would shard by ring pairs and by order m with one all-to-all).  "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1908_00041_amd as vsht
    import vsht_inputs as vi

    L = args.L
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log("grid L=%d" % L)
    xyz, w = vi.gl_grid(L)
    N = len(w)
    a_np, b_np = vi.random_coeffs(L, 0, scale="inv_l")
    K = L * (L + 2)

    # oracle samples (shared by all precisions)
    pidx = vi.sample_indices(N, args.oracle_points, 3)
    cidx = vi.sample_indices(K, args.oracle_coeffs, 4)
    Tr_np = vi.random_field(N, 5)

    results = {}
    for prec in [p for p in args.precisions.split(",") if p]:
        log("precision", prec)
        t_plan = time.perf_counter()
        plan = vsht.Plan(L, xyz, w, precision=prec)
        t_plan = time.perf_counter() - t_plan
        info = plan.info()
        cdt = plan.dtype
        a = torch.from_numpy(a_np).to(dev, cdt)
        b = torch.from_numpy(b_np).to(dev, cdt)
        sec, T, a2, b2 = time_steps(torch, plan, a, b, args.steps, args.warmup)
        log("%s: %.3f ms/step" % (prec, sec * 1e3))
        stages = stage_profile(torch, plan, a, b, max(3, min(args.steps, 10)))
        log("%s stages (ms): %s" % (prec, {k: round(v, 4) for k, v in stages.items()}))
        # errors: round trip (full size), adjoint at sampled points, forward at sampled coeffs
        rt = rel_l2(np.concatenate([a2.cpu().numpy(), b2.cpu().numpy()]),
                    np.concatenate([a_np, b_np]))
        Tg = T.cpu().numpy().astype(np.complex128)
        ga, gb = plan.forward(torch.from_numpy(Tr_np).to(dev, cdt))
        torch.cuda.synchronize()
        results[prec] = dict(sec=sec, stages=stages, roundtrip=rt, T_sample=Tg[pidx],
                             fa=ga.cpu().numpy()[cidx].astype(np.complex128),
                             fb=gb.cpu().numpy()[cidx].astype(np.complex128),
                             plan_s=t_plan, info=info)
        del T, a2, b2, ga, gb
        plan.close()

    l256 = None
    if args.l256:
        l256 = run_l256(torch, vsht, vi, args)
    batched = None
    if args.batch_fields > 0:
        batched = run_batched(torch, vsht, vi, args)
    differentiable = None
    if args.grad_fields > 0:
        differentiable = run_differentiable(torch, vsht, vi, args)
    table3 = run_table3(torch, vsht, vi, args) if args.table3 else None

    if args.copy_mb > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give the
        # scale from counter units to bytes
        src = torch.empty(args.copy_mb * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
        src.fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d MiB" % args.copy_mb)
        del src, dst

    if not results:
        # --precisions "": a run of the other legs alone (for kernel traces); no JSON line
        log("no L=%d precision requested: the other legs ran, no result line" % L)
        return

    cpu = None
    if not args.no_oracle:
        import oracle
        oracle.build(force=False)
        log("oracle: %d coefficients + %d points" % (len(cidx), len(pidx)))
        # the CPU baseline times the first 1024 of each sample (about 15 s of CPU
        # work); the rest of the parity sample runs untimed
        nc, npn = min(len(cidx), 1024), min(len(pidx), 1024)
        t0 = time.perf_counter()
        oa0, ob0 = oracle.forward_subset(L, xyz, w, Tr_np, cidx[:nc])
        t_fwd = time.perf_counter() - t0
        t0 = time.perf_counter()
        oT0 = oracle.adjoint(L, a_np, b_np, xyz[pidx[:npn]])
        t_adj = time.perf_counter() - t0
        oa1, ob1 = oracle.forward_subset(L, xyz, w, Tr_np, cidx[nc:]) if len(cidx) > nc else (oa0[:0], ob0[:0])
        oT1 = oracle.adjoint(L, a_np, b_np, xyz[pidx[npn:]]) if len(pidx) > npn else oT0[:0]
        oa, ob = np.concatenate([oa0, oa1]), np.concatenate([ob0, ob1])
        oT = np.concatenate([oT0, oT1])
        # scale each timed sample to the full transform: forward is linear in the number
        # of coefficients, the adjoint in the number of points
        t_full = t_fwd * K / nc + t_adj * N / npn
        cpu = {"value": 1.0 / t_full, "unit": "transforms/s", "cores": oracle.num_threads(),
               "cpu_model": cpu_model(), "kind": "oracle",
               "sample": ("CPU FP64 direct-sum oracle on the same L=%d GL workload: forward for "
                          "%d sampled coefficients (all %d points, %.2f s) and adjoint at %d "
                          "sampled points (all %d coefficients, %.2f s), each scaled linearly "
                          "to the full transform" % (L, nc, N, t_fwd, npn, 2 * K, t_adj))}
        log("oracle timed sample %.2f s + %.2f s -> %.3g transforms/s" % (t_fwd, t_adj, cpu["value"]))
        for prec, r in results.items():
            r["err_adj"] = rel_l2(r["T_sample"], oT)
            r["err_fwd"] = rel_l2(np.concatenate([r["fa"], r["fb"]]), np.concatenate([oa, ob]))

    peaks = {"fp64": FP64_MFMA_TFLOPS, "fp32": FP32_MFMA_TFLOPS}

    def roofline(prec, r):
        # Dominant kernel of the step and its algorithmic work per launch.
        # Legendre stages: 32 flops per element of E(L) (the method's dense
        # contraction, two functions x eight real columns x multiply-add); BF16x3
        # (BF16x6) performs each multiply-add as 3 (6) bf16 products, counted against
        # the bf16 MFMA peak.  Beside it, the flops this library executes: 16 per
        # element of its spin-frame form (one function, degrees to L+1).  Ring stages:
        # HBM bytes of the field (n x 3 complex) plus the ring-Fourier buffer.
        st = r["stages"]
        dom = max(st, key=lambda k: st[k])
        t = st[dom] * 1e-3
        info = r["info"]
        cs = 16 if prec == "fp64" else 8
        real = "double" if prec == "fp64" else "float"
        nprod = {"bf16x3": 3, "bf16x6": 6}.get(prec, 1)
        # the names the kernel trace shows (ring and coefficient stages: template prefix)
        kern_names = {"leg_fwd": "k_leg_fwd_mfma<%s>" % real, "leg_adj": "k_leg_adj<%s, 0>" % real,
                      "ring_fwd": "k_ring_fwd", "ring_adj": "k_ring_adj",
                      "recombine": "k_recombine", "prep": "k_prep"}
        if nprod > 1:
            kern_names.update(leg_fwd="k_leg_fwd_bf16<%d>" % nprod, leg_adj="k_leg_adj<float, %d>" % nprod)
        kern = kern_names.get(dom, dom)
        out = {"kernel": kern, "launch_us": round(st[dom] * 1e3, 2)}
        if dom in ("leg_fwd", "leg_adj"):
            flops = 32.0 * nprod * method_elements(L)
            executed = 16.0 * nprod * folded_elements(L, info["n_pairs"])
            peak = peaks.get(prec, BF16_MFMA_TFLOPS)
            # the binary64 and binary32 plans' synthesis runs in binary64 on the vector
            # unit: its peak is the binary64 vector rate (78.6 TFLOP/s, equal to the
            # binary64 matrix-core peak)
            bound = "mfma"
            if dom == "leg_adj" and nprod == 1:
                bound, peak = "alu", FP64_MFMA_TFLOPS
            ach = flops / t / 1e12
            out.update(bound=bound, achieved=round(ach, 3), peak=peak, unit="TFLOP/s",
                       frac=round(ach / peak, 4), flops_per_launch=flops,
                       executed_flops_per_launch=executed,
                       executed_frac=round(executed / t / 1e12 / peak, 4))
        else:
            nbuf = (L + 1) * (info["n_rings"] * 4 if dom == "ring_fwd" else info["n_pairs"] * 8)
            if dom in ("ring_fwd", "ring_adj"):
                by = (3 * N + nbuf) * cs
            else:  # coefficient stages: 2K coefficients and the (L+2)-row triangle
                by = (2 * K + 4 * (L + 1) * (L + 4) // 2) * cs
            ach = by / t / 1e9
            out.update(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                       frac=round(ach / HBM_PEAK_GBS, 4), bytes_per_launch=by)
        out["traffic"] = measured_traffic(kern, prec, L)
        return out

    def step_roofline(prec, r):
        # the whole forward+adjoint step: t_roof = max(compulsory bytes / HBM peak,
        # the method's Legendre flops / the precision's peak); frac = t_roof / t_step
        cs = 16 if prec == "fp64" else 8
        nprod = {"bf16x3": 3, "bf16x6": 6}.get(prec, 1)
        by = 2.0 * (3 * N + 2 * K) * cs
        fl = 64.0 * nprod * method_elements(L)
        t_hbm = by / (HBM_PEAK_GBS * 1e9)
        t_fl = fl / (peaks.get(prec, BF16_MFMA_TFLOPS) * 1e12)
        t_roof = max(t_hbm, t_fl)
        return {"bound": "hbm" if t_hbm >= t_fl else "compute",
                "bytes": by, "flops": fl, "t_roof_us": round(t_roof * 1e6, 2),
                "t_step_us": round(r["sec"] * 1e6, 2), "frac": round(t_roof / r["sec"], 4)}

    main_r = results.get("fp64") or next(iter(results.values()))
    main_prec = "fp64" if "fp64" in results else next(iter(results))
    ms = main_r["sec"] * 1e3
    out = {
        "metric": "VSHT fwd+adj transforms/s at L=1024 + % HBM/MFMA roofline, at stated error vs FP64",
        "value": round(1.0 / main_r["sec"], 2),
        "unit": "transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32"}.get(main_prec, main_prec + "/f32"),
        "data": "synthetic",
        "config": {"workload": "forward+adjoint VSHT, Gauss-Legendre grid %dx%d (%d points), "
                               "L=%d, random coefficients scaled 1/l, seed 0" % (L + 1, 2 * L + 2, N, L),
                   "L": L, "points": N, "coefficients": 2 * K, "precision": main_prec},
        "roofline": roofline(main_prec, main_r),
        "step_roofline": step_roofline(main_prec, main_r),
        "plan_s": round(main_r["plan_s"], 3),
        "stages_us": {k: round(v * 1e3, 2) for k, v in main_r["stages"].items()},
        "errors": {"roundtrip_rel_l2": main_r["roundtrip"]},
        "cpu_baseline": cpu,
    }
    if "err_adj" in main_r:
        out["errors"].update(adjoint_vs_oracle_rel_l2=main_r["err_adj"],
                             forward_vs_oracle_rel_l2=main_r["err_fwd"],
                             oracle_sample={"coefficients": int(len(cidx)), "points": int(len(pidx))})
    variants = {}
    for prec, r in results.items():
        if prec == main_prec:
            continue
        v = {"value": round(1.0 / r["sec"], 2), "ms_per_step": round(r["sec"] * 1e3, 4),
             "roofline": roofline(prec, r), "step_roofline": step_roofline(prec, r),
             "plan_s": round(r["plan_s"], 3),
             "stages_us": {k: round(x * 1e3, 2) for k, x in r["stages"].items()},
             "errors": {"roundtrip_rel_l2": r["roundtrip"]}}
        if "err_adj" in r:
            v["errors"].update(adjoint_vs_oracle_rel_l2=r["err_adj"],
                               forward_vs_oracle_rel_l2=r["err_fwd"])
        variants[prec] = v
    if variants:
        out["variants"] = variants
    if l256:
        out["L256"] = l256
    if batched:
        out["batched"] = batched
    if differentiable:
        out["differentiable"] = differentiable
    if table3:
        out["table3"] = table3
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
