#!/usr/bin/env python3
"""Benchmark of the XCT hot path on one MI355X.

Workload (the paper-shaped batch the headline metric is quoted on): 16 slices
of 1024 x 1024 voxels, 1500 angles over [0, pi), 1024 channels, one shared
Siddon matrix; seeded 40-ellipsoid phantom, synthetic data.

A step is one forward projection y = A x plus one backprojection x = A^T y
of the whole 16-slice batch through the C ABI (FP32 path: matrix values FP32
with 16-bit stage-local indices, FP32 vectors), with inputs resident in HBM.
`value` is the algorithmic bytes of a step per second (GB/s):
  per product  ceil(B/F) * nnz * b_A  +  B * (n_in + n_out) * 4
with b_A = 6 (u16 slot + f32 length), n_in/n_out = N^2 and M*C.
The roofline object covers the SpMM kernel (both operators are launches of
the same kernel): its algorithmic bytes per launch divided by its launch
durations, measured with HIP events on the launch stream.

Also reported: CGLS seconds per iteration for the FP32 matrix and for the
FP16 matrix (16-bit storage of matrix values and kernel operands, FP32
accumulation), and the FP64 CPU oracle timed on a bounded sample of the same
products on the host cores.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "fwd+back projection GB/s & % HBM peak; CGLS s/iter, FP16-store vs FP32"


def alg_bytes(nnz, n_in, n_out, B, F, b_a, b_vec=4):
    return math.ceil(B / F) * nnz * b_a + B * (n_in + n_out) * b_vec


def measured_traffic(dtype, N, M, B, default_opts):
    """HBM bytes per SpMM launch from the committed rocprofv3 counter summary of
    this workload, if it was taken on the current kernel sources; else None."""
    from paper_2009_07226_amd import pmc_summary
    path = os.path.join(ROOT, "profiles", f"k_spmm_traffic_{dtype}_{B}x{N}x{M}.json")
    if not default_opts or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_sources_sha256") != pmc_summary.kernel_sources_sha():
        return None
    ks = list(rec["kernels"].values())
    n = sum(k["launches"] for k in ks)
    tot = sum((k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]) * k["launches"] for k in ks)
    return tot / n if n else None


def cpu_baseline(N, M, C, B, x_host, bytes_step, budget_s):
    """FP64 oracle (matrix-free sampled rows of A and voxels of A^T) on the host cores."""
    import numpy as np

    import oracle

    rng = np.random.default_rng(0)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    oracle.set_threads(threads)
    ys = rng.random((B, M * C))

    def rate(fn, total, n0):
        idx = rng.choice(total, n0, replace=False)
        t = time.perf_counter()
        fn(idx)
        return n0 / (time.perf_counter() - t)

    fr = lambda idx: oracle.project_rows(N, M, C, x_host, idx)
    fb = lambda idx: oracle.backproject_voxels(N, M, C, ys, idx)
    # calibrate, then time a sample sized to about budget_s of CPU work
    r_rows = rate(fr, M * C, 256)
    r_vox = rate(fb, N * N, 256)
    n_rows = int(min(M * C, max(512, r_rows * budget_s / 2)))
    n_vox = int(min(N * N, max(512, r_vox * budget_s / 2)))
    r_rows = rate(fr, M * C, n_rows)
    r_vox = rate(fb, N * N, n_vox)
    t_full = M * C / r_rows + N * N / r_vox
    return {
        "value": bytes_step / t_full / 1e9,
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"FP64 oracle, matrix-free: {n_rows} random rays of A and {n_vox} random voxels of A^T, "
                   f"each over all {B} slices; full-step time extrapolated linearly "
                   f"({t_full:.1f} s per fwd+back step)"),
        "s_per_step": t_full,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cgls-iters", type=int, default=30)
    ap.add_argument("--no-cgls", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--angles", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--stage-order", type=int, default=0, help="0 sweep (default), 1 Hilbert")
    ap.add_argument("--lds-bytes", type=int, default=0)
    ap.add_argument("--tile-waves", type=int, default=0)
    ap.add_argument("--lane-order", type=int, default=0)
    ap.add_argument("--slab-order", type=int, default=0)
    ap.add_argument("--fuse", type=int, default=0, help="slices fused per matrix pass (1, 2, 4, 8, 16; default 16)")
    ap.add_argument("--arith", type=int, default=0,
                    help="1: FP16 arithmetic for the FP16 matrices (the paper's half-precision variant)")
    ap.add_argument("--streamed", type=int, default=0, metavar="BATCH",
                    help="also time a step over BATCH host-resident slices (streamed entry points, chunks of "
                         "fuse slices, PCIe-inclusive)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (reference for profiler byte counters)")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16"],
                    help="matrix/operand storage of the timed projection step (FP32 is the headline path)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2009_07226_amd as xct
    from paper_2009_07226_amd import gradient as pgrad
    from paper_2009_07226_amd import phantoms

    N, M, C, B = args.n, args.angles, args.n, args.batch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    log(f"building {args.dtype} matrix N={N} M={M} C={C}")
    opts = dict(stage_order=args.stage_order, lds_bytes=args.lds_bytes, tile_waves=args.tile_waves, fuse=args.fuse,
                lane_order=args.lane_order, slab_order=args.slab_order)
    opts16 = dict(opts, arith=args.arith)  # FP16 arithmetic applies to FP16 matrices only
    A = xct.Matrix(N, M, C, args.dtype, **(opts16 if args.dtype == "f16" else opts))
    b_a = 6 if args.dtype == "f32" else 4
    b_x = 4 if args.dtype == "f32" else 2
    info = A.info()
    log(f"built in {info['build_seconds']:.2f} s: A nnz {info['A']['nnz']:,} padded {info['A']['padded']:,}; "
        f"A^T padded {info['AT']['padded']:,}")
    F = min(int(info["fuse"]), 1 << max(0, (B - 1).bit_length()))  # slices per matrix pass
    nnz = info["A"]["nnz"]
    bytes_A = alg_bytes(nnz, N * N, M * C, B, F, b_a)
    bytes_AT = alg_bytes(info["AT"]["nnz"], M * C, N * N, B, F, b_a)
    bytes_step = bytes_A + bytes_AT

    x = phantoms.ellipsoid_phantom(N, B, 40, seed=2, device=dev).float()
    y = torch.empty((B, M, C), dtype=torch.float32, device=dev)
    xb = torch.empty((B, N, N), dtype=torch.float32, device=dev)
    ws = A.spmm_workspace(B)

    def step():
        xct.project(A, x, out=y, workspace=ws)
        xct.backproject(A, y, out=xb, workspace=ws)

    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nb} bytes read, {nb} bytes written")
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    xct.profile_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    xct.profile_enable(False)
    prof = xct.profile_read()
    ms_step = e0.elapsed_time(e1) / args.steps
    value = bytes_step / (ms_step * 1e-3) / 1e9
    nA, msA = prof["A"]
    nT, msT = prof["AT"]
    # kernel: matrix entries + staged operand (storage dtype) in + FP32 sums out
    kern_bytes_A = nnz * b_a + F * (N * N * b_x + M * C * 4)
    kern_bytes_AT = info["AT"]["nnz"] * b_a + F * (M * C * b_x + N * N * 4)
    launches = nA + nT
    avg_ms = (msA + msT) / max(launches, 1)
    achieved = (kern_bytes_A * nA + kern_bytes_AT * nT) / ((msA + msT) * 1e-3) / 1e9
    log(f"step {ms_step:.3f} ms ({wall / args.steps * 1e3:.3f} ms wall), {value:.1f} GB/s; "
        f"SpMM A {msA / max(nA, 1):.3f} ms, A^T {msT / max(nT, 1):.3f} ms per launch")

    # context: what a plain streaming read (16-byte non-temporal loads) reaches
    # on this device over 4 GiB resident in HBM
    big = torch.ones(1 << 30, dtype=torch.float32, device=dev)
    read_ceiling = xct.read_bandwidth(big, reps=5)
    del big
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"{B} slices {N}x{N}, {M} angles over [0,pi), {C} channels, shared Siddon "
                               f"matrix ({args.dtype} values, 16-bit stage-local indices); 40-ellipsoid phantom",
                   "n": N, "angles": M, "channels": C, "batch": B, "fuse": F},
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "read_ceiling_GBps": round(read_ceiling, 1),
        "pct_of_read_ceiling": round(100.0 * value / read_ceiling, 2),
        "slice_nnz_per_s": (nnz + info["AT"]["nnz"]) * B / (ms_step * 1e-3),
        "nnz": nnz,
        "padded_A": info["A"]["padded"],
        "padded_AT": info["AT"]["padded"],
        "padding_ratio": round((info["A"]["padded"] + info["AT"]["padded"]) / (nnz + info["AT"]["nnz"]), 4),
        "balanced_slabs": [info["A"]["balanced_slabs"], info["A"]["slabs"], info["AT"]["balanced_slabs"],
                           info["AT"]["slabs"]],
        "build_s_f32": round(info["build_seconds"], 3),
        "plan": {"stages_A": info["A"]["stages"], "stages_AT": info["AT"]["stages"],
                 "tiles_per_stage": info["A"]["tiles_per_stage"], "blocks_A": info["A"]["blocks"],
                 "blocks_AT": info["AT"]["blocks"], "staged_slots_A": info["A"]["staged_slots"],
                 "staged_slots_AT": info["AT"]["staged_slots"], "stage_order": args.stage_order},
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_spmm<{args.dtype},{F}> (A and A^T launches)",
            "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(args.dtype, N, M, B,
                                        not (args.stage_order or args.lds_bytes or args.tile_waves or args.fuse or
                                             args.arith or
                                             args.lane_order or args.slab_order)),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "avg_launch_ms": round(avg_ms, 4),
            "alg_bytes_per_launch": {"A": kern_bytes_A, "AT": kern_bytes_AT},
            "launch_ms": {"A": round(msA / max(nA, 1), 4), "AT": round(msT / max(nT, 1), 4)},
        },
    }

    if args.streamed:
        # host-resident batch (the benchmark batch repeated): chunks of F slices
        # copied in and out on two copy streams while the SpMM runs;
        # PCIe-inclusive, never the headline value
        BS = args.streamed
        log(f"streamed step ({BS} host-resident slices)")
        xh = x.cpu().repeat((BS + B - 1) // B, 1, 1)[:BS].contiguous().pin_memory()
        yh = torch.empty((BS, M, C), dtype=torch.float32, pin_memory=True)
        xbh = torch.empty((BS, N, N), dtype=torch.float32, pin_memory=True)
        ws_p = torch.empty(xct.lib().xct_stream_workspace_bytes(A.handle, 0, F, 0), dtype=torch.uint8, device=dev)
        ws_b = torch.empty(xct.lib().xct_stream_workspace_bytes(A.handle, 1, F, 0), dtype=torch.uint8, device=dev)
        for _ in range(2):
            xct.project_streamed(A, xh, out=yh, chunk=F, workspace=ws_p)
            xct.backproject_streamed(A, yh, out=xbh, chunk=F, workspace=ws_b)
        ts = time.perf_counter()
        for _ in range(args.steps):
            xct.project_streamed(A, xh, out=yh, chunk=F, workspace=ws_p)
            xct.backproject_streamed(A, yh, out=xbh, chunk=F, workspace=ws_b)
        ms_s = (time.perf_counter() - ts) / args.steps * 1e3
        bytes_s = (alg_bytes(nnz, N * N, M * C, BS, F, b_a) +
                   alg_bytes(info["AT"]["nnz"], M * C, N * N, BS, F, b_a))
        host_bytes = 2 * BS * (N * N + M * C) * 4  # each step copies x and y in and out once
        out["streamed_step"] = {"batch": BS, "chunk": F, "ms_per_step": round(ms_s, 3),
                                "GBps": round(bytes_s / (ms_s * 1e-3) / 1e9, 2),
                                "device_resident_equivalent_ms": round(ms_step * math.ceil(BS / B), 3),
                                "host_bytes_per_step": host_bytes,
                                "host_GBps": round(host_bytes / (ms_s * 1e-3) / 1e9, 2),
                                "note": "PCIe-inclusive; slices resident in pinned host memory"}
        log(f"streamed step {ms_s:.3f} ms")
        del xh, yh, xbh, ws_p, ws_b

    if not args.no_cgls:
        it = args.cgls_iters
        yc = (y + 0.01 * float(y.abs().max()) * phantoms.noise_torch((M, C), B, 2, dev)).contiguous()

        def cgls_time(Am, iters, reps=2):
            wsc = Am.cgls_workspace(B, iters)
            xo = torch.empty((B, N, N), dtype=torch.float32, device=dev)
            xct.cgls(Am, yc, iters, out=xo, workspace=wsc, want_resid=False)
            torch.cuda.synchronize()
            best = float("inf")
            for _ in range(reps):
                s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s0.record()
                xct.cgls(Am, yc, iters, out=xo, workspace=wsc, want_resid=False)
                s1.record()
                torch.cuda.synchronize()
                best = min(best, s0.elapsed_time(s1) * 1e-3)
            return best

        def cgls_history(Am):
            # untimed run with the per-iteration residual history ||y - A x_k|| / ||y||
            xo, res, _ = xct.cgls(Am, yc, it)
            return xo, res

        checkpoints = [k for k in (0, 1, 2, 3, 5, 10, 20, 30, 50) if k <= it]
        log("CGLS FP32")
        A32 = A if args.dtype == "f32" else xct.Matrix(N, M, C, "f32", **opts)
        t32 = (cgls_time(A32, it) - cgls_time(A32, 0)) / it
        x32, res32 = cgls_history(A32)
        del A32
        if args.dtype == "f32":
            del A
        torch.cuda.empty_cache()
        log("building FP16 matrix")
        A16 = A if args.dtype == "f16" else xct.Matrix(N, M, C, "f16", **opts16)
        log("CGLS FP16 storage")
        t16 = (cgls_time(A16, it) - cgls_time(A16, 0)) / it
        x16, res16 = cgls_history(A16)
        d16 = ((x16 - x32).flatten(1).norm(dim=1) / x32.flatten(1).norm(dim=1).clamp_min(1e-30)).max().item()
        del x32, x16
        # the FP16 operators' projection + backprojection step, for reference
        i16 = A16.info()
        ws16 = A16.spmm_workspace(B)
        for _ in range(2):
            xct.project(A16, x, out=y, workspace=ws16)
        torch.cuda.synchronize()
        xct.profile_enable(True)
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record()
        for _ in range(args.steps):
            xct.project(A16, x, out=y, workspace=ws16)
            xct.backproject(A16, y, out=xb, workspace=ws16)
        f1.record()
        torch.cuda.synchronize()
        xct.profile_enable(False)
        p16 = xct.profile_read()
        ms16 = f0.elapsed_time(f1) / args.steps
        kb16 = {w: i16[w]["nnz"] * 4 + F * (N * N * 2 + M * C * 4) for w in ("A", "AT")}
        ach16 = (kb16["A"] * p16["A"][0] + kb16["AT"] * p16["AT"][0]) / ((p16["A"][1] + p16["AT"][1]) * 1e-3) / 1e9
        b16 = alg_bytes(i16["A"]["nnz"], N * N, M * C, B, F, 4) + alg_bytes(i16["AT"]["nnz"], M * C, N * N, B, F, 4)
        out["fp16_step"] = {"ms_per_step": round(ms16, 4), "GBps": round(b16 / (ms16 * 1e-3) / 1e9, 2),
                            "kernel_GBps": round(ach16, 2), "kernel_frac": round(ach16 / HBM_PEAK_GBS, 4),
                            "launch_ms": {"A": round(p16["A"][1] / max(p16["A"][0], 1), 4),
                                          "AT": round(p16["AT"][1] / max(p16["AT"][0], 1), 4)},
                            "padded_A": i16["A"]["padded"], "padded_AT": i16["AT"]["padded"]}
        # convergence against time: median relative residual over the slices
        # after k iterations, reached at k * s/iter
        out["cgls"] = {"iters": it, "fp32_s_per_iter": round(t32, 6), "fp16_s_per_iter": round(t16, 6),
                       "fp16_speedup": round(t32 / t16, 3),
                       "residual_median": {"k": checkpoints,
                                           "fp32": [float(np.median(res32[k])) for k in checkpoints],
                                           "fp16": [float(np.median(res16[k])) for k in checkpoints]},
                       "fp16_vs_fp32_rel_l2_max": round(d16, 6),
                       "build_s_f16": round(A16.info()["build_seconds"], 3)}
        log(f"CGLS s/iter FP32 {t32 * 1e3:.3f} ms, FP16 {t16 * 1e3:.3f} ms")
        # the generic gradient solver of Eq. (1) (x >= 0, TV) on the same
        # FP16 operators: torch autograd around the projection pair
        log("projected gradient FP16")
        lam, eps, pg_it = 0.1, 0.05, 5
        tau = 0.95 / pgrad.lipschitz(A16, lam, eps, 10)
        pgrad.projected_gradient(A16, yc, 1, tau, lam=lam, eps=eps)
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record()
        pgrad.projected_gradient(A16, yc, pg_it, tau, lam=lam, eps=eps)
        g1.record()
        torch.cuda.synchronize()
        tpg = g0.elapsed_time(g1) * 1e-3 / pg_it
        out["projected_gradient"] = {"iters": pg_it, "lam": lam, "eps": eps, "fp16_s_per_iter": round(tpg, 6),
                                     "vs_spmm_pair": round(tpg / (ms16 * 1e-3), 3)}
        del A16

    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(N, M, C, B, x.double().cpu().numpy().reshape(B, -1), bytes_step,
                                           args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
