#!/usr/bin/env python3
"""Benchmark of the XCT hot path on one MI355X.

Headline workload (the paper-shaped batch the headline metric is quoted on):
16 slices of 1024 x 1024 voxels, 1500 angles over [0, pi), 1024 channels, one
shared Siddon matrix; seeded 40-ellipsoid phantom, synthetic data.

A step is one forward projection y = A x plus one backprojection x = A^T y
of the whole 16-slice batch through the C ABI (FP32 path: matrix values FP32
with 16-bit stage-local indices, FP32 vectors), with inputs resident in HBM.
`value` is the algorithmic bytes of a step per second (GB/s):
  per product  ceil(B/F) * nnz * b_A  +  B * (n_in + n_out) * 4
with b_A = 6 (u16 slot + f32 length), n_in/n_out = N^2 and M*C.
The roofline object covers the SpMM kernel (both operators are launches of
the same kernel): its algorithmic bytes per launch divided by its launch
durations, measured with HIP events on the launch stream.

Also reported (each in its own object of the JSON line):
  * CGLS seconds per iteration for the FP32 matrix and for the FP16 matrix
    (16-bit storage of matrix values and kernel operands, FP32 accumulation);
  * the 64 x 2048^2 x 1500 batch (FP32, FP16, BF16: kernel share of the HBM
    peak, step and CGLS s/iter) and the 128 x 2816^2 x 2250 share (FP16:
    kernel share, 20 CGLS iterations);
  * the CPU oracle leg: the FP64 oracle timed on a bounded sample of the
    headline products on the host cores (all cores and one core, median of
    three), and the relative errors of the GPU outputs against the oracle:
    sampled rays and voxels of the headline products, CGLS per iteration
    (FP32, FP16, BF16) on 2 slices of 512^2 x 360 over 30 iterations and on 2
    slices of 2048^2 x 1500 over the first 3 iterations.
"""
import argparse
import json
import math
import os
import subprocess
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "fwd+back projection GB/s & % HBM peak; CGLS s/iter, FP16-store vs FP32"
BYTES_A = {"f32": 6, "f16": 4, "bf16": 4, "f64": 10}  # stored bytes per matrix entry
BYTES_X = {"f32": 4, "f16": 2, "bf16": 2, "f64": 8}   # staged operand bytes per element
BYTES_Y = {"f32": 4, "f16": 4, "bf16": 4, "f64": 8}   # sums written per output element


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


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


# ---- GPU measurements -----------------------------------------------------------

def time_products(xct, torch, A, x, steps, warmup=2):
    """Projection + backprojection of the batch x, `steps` times: ms per step
    and, from the library's launch events, the SpMM kernel's launch times and
    its algorithmic byte rate (matrix entries + staged operand in + FP32 out)."""
    info = A.info()
    dt = {0: "f32", 1: "f16", 2: "bf16", 3: "f64"}[info["value_dtype"]]
    B, N, M, C = x.shape[0], A.n, A.n_angles, A.n_channels
    F = min(int(info["fuse"]), 1 << max(0, (B - 1).bit_length()))
    y = torch.empty((B, M, C), dtype=x.dtype, device=x.device)
    xb = torch.empty_like(x)
    ws = A.spmm_workspace(B)
    for _ in range(warmup):
        xct.project(A, x, out=y, workspace=ws)
        xct.backproject(A, y, out=xb, workspace=ws)
    torch.cuda.synchronize()
    xct.profile_enable(True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        xct.project(A, x, out=y, workspace=ws)
        xct.backproject(A, y, out=xb, workspace=ws)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    xct.profile_enable(False)
    prof = xct.profile_read()
    ms = e0.elapsed_time(e1) / steps
    b_a, b_x, b_y = BYTES_A[dt], BYTES_X[dt], BYTES_Y[dt]
    nnzA, nnzT = info["A"]["nnz"], info["AT"]["nnz"]
    kb = {"A": nnzA * b_a + F * (N * N * b_x + M * C * b_y), "AT": nnzT * b_a + F * (M * C * b_x + N * N * b_y)}
    (nA, msA), (nT, msT) = prof["A"], prof["AT"]
    ach = (kb["A"] * nA + kb["AT"] * nT) / ((msA + msT) * 1e-3) / 1e9
    b_io = x.element_size()
    step_bytes = alg_bytes(nnzA, N * N, M * C, B, F, b_a, b_io) + alg_bytes(nnzT, M * C, N * N, B, F, b_a, b_io)
    del y, xb, ws
    return {"dtype": dt, "fuse": F, "ms_per_step": round(ms, 4), "wall_ms_per_step": round(wall / steps * 1e3, 4),
            "GBps": round(step_bytes / (ms * 1e-3) / 1e9, 2), "bytes_step": step_bytes,
            "kernel_GBps": round(ach, 2), "kernel_frac": round(ach / HBM_PEAK_GBS, 4),
            "avg_launch_ms": round((msA + msT) / max(nA + nT, 1), 4),
            "launch_ms": {"A": round(msA / max(nA, 1), 4), "AT": round(msT / max(nT, 1), 4)},
            "alg_bytes_per_launch": kb, "nnz": nnzA, "padded_A": info["A"]["padded"],
            "padded_AT": info["AT"]["padded"], "build_s": round(info["build_seconds"], 3)}


def cgls_seconds(xct, torch, A, y, iters, reps=2):
    """Best of `reps` timed CGLS runs of `iters` iterations (no residual copy)."""
    B = y.shape[0]
    wsc = A.cgls_workspace(B, iters)
    xo = torch.empty((B, A.n, A.n), dtype=torch.float32, device=y.device)
    xct.cgls(A, y, iters, out=xo, workspace=wsc, want_resid=False)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record()
        xct.cgls(A, y, iters, out=xo, workspace=wsc, want_resid=False)
        s1.record()
        torch.cuda.synchronize()
        best = min(best, s0.elapsed_time(s1) * 1e-3)
    return best


def cgls_s_per_iter(xct, torch, A, y, iters):
    """(t(iters) - t(0)) / iters: the setup backprojection excluded."""
    return (cgls_seconds(xct, torch, A, y, iters) - cgls_seconds(xct, torch, A, y, 0)) / iters


def gpu_cgls_iterates(xct, A, y, K):
    """x_1..x_K of the GPU CGLS as a host FP64 array (K, B, cols), one run per
    k (the solver is deterministic), and the K-run's residual history."""
    import numpy as np
    xs = []
    res = None
    for k in range(1, K + 1):
        x, res, _ = xct.cgls(A, y, k)
        xs.append(x.double().cpu().numpy().reshape(y.shape[0], -1))
    return np.stack(xs), res


# ---- the CPU oracle leg (the FP64 oracle: timing and errors) ---------------------

def rel_l2_rows(a, b):
    import numpy as np
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def per_iteration_errors(xg, xo):
    """max over slices of ||x_k - x_k*|| / ||x_k*||, k = 1..K"""
    return [float(rel_l2_rows(xg[k], xo[k]).max()) for k in range(xg.shape[0])]


def holds_through(errs, bar):
    """last k such that every iterate up to k is within `bar` (0: not even x_1)"""
    k = 0
    for e in errs:
        if e > bar:
            break
        k += 1
    return k


def cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return "unknown"


def cpu_baseline(oracle, N, M, C, B, x_host, ys, bytes_step, budget_s, threads):
    """The FP64 oracle (matrix-free: sampled rows of A and voxels of A^T over
    all B slices) on the host cores: a calibration, then three samples sized
    to about budget_s / 4 each at all cores (median reported) and one at a
    single core; full-step time extrapolated linearly in rows and voxels."""
    import numpy as np
    rng = np.random.default_rng(0)

    def rates(n_rows, n_vox):
        ir = rng.choice(M * C, n_rows, replace=False)
        iv = rng.choice(N * N, n_vox, replace=False)
        t = time.perf_counter()
        oracle.project_rows(N, M, C, x_host, ir)
        tr = time.perf_counter() - t
        t = time.perf_counter()
        oracle.backproject_voxels(N, M, C, ys, iv)
        tv = time.perf_counter() - t
        return n_rows / tr, n_vox / tv

    oracle.set_threads(threads)
    r_rows, r_vox = rates(256, 256)  # calibration (also the warm-up)
    per = budget_s / 4.0
    n_rows = int(min(M * C, max(512, r_rows * per / 2)))
    n_vox = int(min(N * N, max(512, r_vox * per / 2)))
    t_full = []
    for _ in range(3):
        rr, rv = rates(n_rows, n_vox)
        t_full.append(M * C / rr + N * N / rv)
    t_med = float(np.median(t_full))
    oracle.set_threads(1)
    n1r, n1v = max(64, n_rows // threads), max(64, n_vox // threads)
    rr, rv = rates(n1r, n1v)
    t_one = M * C / rr + N * N / rv
    oracle.set_threads(threads)
    return {
        "value": bytes_step / t_med / 1e9,
        "unit": "GB/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"FP64 oracle, matrix-free: {n_rows} random rays of A and {n_vox} random voxels of A^T, "
                   f"each over all {B} slices, on {threads} threads, median of 3 after a calibration run; "
                   f"full-step time extrapolated linearly ({t_med:.1f} s per fwd+back step); one core: "
                   f"{n1r} rays and {n1v} voxels"),
        "s_per_step": t_med,
        "s_per_step_runs": [round(t, 3) for t in t_full],
        "one_core": {"value": bytes_step / t_one / 1e9, "unit": "GB/s", "s_per_step": t_one},
    }


def headline_errors(oracle, xct, torch, A, N, M, C, x, y, slices, seed=7, n=512):
    """Relative L2 (max over the listed slices) of the headline products on
    sampled outputs: rays of A x (y the GPU projection of x) and voxels of
    A^T w for a seeded uniform random sinogram w."""
    import numpy as np
    rng = np.random.default_rng(seed)
    rows = rng.choice(M * C, n, replace=False)
    vox = rng.choice(N * N, n, replace=False)
    xs = x[slices].double().cpu().numpy().reshape(len(slices), -1)
    ref = oracle.project_rows(N, M, C, xs, rows)
    got = y[slices].reshape(len(slices), -1)[:, torch.from_numpy(rows).to(y.device)].double().cpu().numpy()
    e_p = float(rel_l2_rows(got, ref).max())
    w = torch.rand(y.shape, generator=torch.Generator().manual_seed(seed), dtype=torch.float32)
    xb = xct.backproject(A, w.to(y.device))
    ref = oracle.backproject_voxels(N, M, C, w[slices].double().numpy(), vox)
    got = xb[slices].reshape(len(slices), -1)[:, torch.from_numpy(vox).to(y.device)].double().cpu().numpy()
    e_b = float(rel_l2_rows(got, ref).max())
    return {"projection_rel_l2": e_p, "backprojection_rel_l2": e_b, "slices": list(slices),
            "samples": f"{n} random rays of A x and {n} random voxels of A^T w (w: seeded uniform sinogram), "
                       "traced by the oracle"}


def product_errors(oracle, xct, torch, A, x, slices, seed=11, n=256):
    """Sampled errors of one matrix's products on the listed slices of x (the
    timed batch): n random rays of A x and n random voxels of A^T w (w a
    seeded uniform sinogram), each traced by the oracle."""
    import numpy as np
    N, M, C = A.n, A.n_angles, A.n_channels
    xs = x[slices].contiguous()
    w = torch.rand((len(slices), M, C), generator=torch.Generator().manual_seed(seed), dtype=torch.float32)
    y = xct.project(A, xs)
    xb = xct.backproject(A, w.to(x.device).to(x.dtype))
    rng = np.random.default_rng(seed)
    rows = rng.choice(M * C, n, replace=False)
    vox = rng.choice(N * N, n, replace=False)
    ref = oracle.project_rows(N, M, C, xs.double().cpu().numpy().reshape(len(slices), -1), rows)
    got = y.reshape(len(slices), -1)[:, torch.from_numpy(rows).to(y.device)].double().cpu().numpy()
    e_p = float(rel_l2_rows(got, ref).max())
    ref = oracle.backproject_voxels(N, M, C, w.double().numpy(), vox)
    got = xb.reshape(len(slices), -1)[:, torch.from_numpy(vox).to(xb.device)].double().cpu().numpy()
    e_b = float(rel_l2_rows(got, ref).max())
    return {"projection_rel_l2": round(e_p, 9), "backprojection_rel_l2": round(e_b, 9), "slices": list(slices),
            "samples": n}


def cgls_errors_512(oracle, xct, torch, phantoms, dev, iters=30):
    """CGLS iterates of the three storage formats against the oracle's, every
    iteration, on 2 slices of 512^2 x 360 (1% noise)."""
    N, M, C = 512, 360, 512
    Ao, ATo = oracle.build_A(N, M, C), oracle.build_AT(N, M, C)
    x_true = phantoms.ellipsoid_phantom(N, 8, 20, seed=3)[[2, 5]]
    y = oracle.project(Ao, x_true.numpy().reshape(2, -1))
    y = y + 0.01 * y.max() * phantoms.noise((M * C,), [2, 5], 3)
    y32 = torch.from_numpy(y).float().reshape(2, M, C)
    _, reso, _, xho = oracle.cgls(Ao, ATo, y32.double().numpy().reshape(2, -1), iters, history=True)
    out = {"workload": "2 slices 512x512, 360 angles, 512 channels, 20-ellipsoid phantom, 1% noise",
           "k": list(range(1, iters + 1))}
    for dt in ("f32", "f16", "bf16"):
        A = xct.Matrix(N, M, C, dt)
        xg, resg = gpu_cgls_iterates(xct, A, y32.to(dev), iters)
        out[dt] = [round(e, 8) for e in per_iteration_errors(xg, xho)]
        out[dt + "_residual_rel_dev_max"] = float((abs(resg - reso) / reso).max())
        A.free()
    out["f32_within_1e-4_through_k"] = holds_through(out["f32"], 1e-4)
    out["f16_within_1e-3_through_k"] = holds_through(out["f16"], 1e-3)
    out["bf16_within_1e-3_through_k"] = holds_through(out["bf16"], 1e-3)
    return out


class TracedOracleCgls(threading.Thread):
    """The oracle's CGLS history on a few slices of a scan too large for an
    explicit A and A^T in host memory (A traced into a CSR, A^T applied as its
    transposed product), run on the host while the GPU measurements go on.
    The sinogram is the oracle's projection of the phantom slices x (FP64)
    plus 1% seeded noise, rounded to FP32; ``sinogram()`` waits for it and
    returns it for the GPU side, so both solve the same problem."""

    def __init__(self, oracle, phantoms, N, M, C, x, slices, seed, iters, threads):
        super().__init__(daemon=True)
        self.args = (oracle, phantoms, N, M, C, x, slices, seed, iters, threads)
        self.result, self.error, self.seconds, self.y = None, None, None, None
        self._y_ready = threading.Event()

    def sinogram(self):
        self._y_ready.wait()
        return self.y

    def run(self):
        import numpy as np
        oracle, phantoms, N, M, C, x, slices, seed, iters, threads = self.args
        t = time.perf_counter()
        try:
            oracle.set_threads(threads)
            with oracle.TracedA(N, M, C) as T:
                y = T.project(x)
                y = y + 0.01 * np.abs(y).max() * phantoms.noise((M * C,), slices, seed)
                self.y = y.astype(np.float32).astype(np.float64)
                self._y_ready.set()
                _, res, _, xh = T.cgls(self.y, iters, history=True)
            self.result = (xh, res)
        except Exception as e:  # reported in the JSON line, never raised from the thread
            self.error = repr(e)
        finally:
            self._y_ready.set()
        self.seconds = time.perf_counter() - t


# ---- main ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cgls-iters", type=int, default=30)
    ap.add_argument("--no-cgls", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg (timing and errors)")
    ap.add_argument("--no-large", action="store_true", help="skip the 64 x 2048^2 and 128 x 2816^2 workloads")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--angles", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--stage-order", type=int, default=0, help="0 sweep (default), 1 Hilbert")
    ap.add_argument("--lds-bytes", type=int, default=0)
    ap.add_argument("--tile-waves", type=int, default=0)
    ap.add_argument("--lane-order", type=int, default=0)
    ap.add_argument("--slab-order", type=int, default=0)
    ap.add_argument("--xcd-remap", type=int, default=0,
                    help="workgroup-to-XCD mapping: runs of n blocks (0: default 4), 1 contiguous, -1 plain")
    ap.add_argument("--fuse", type=int, default=0,
                    help="slices fused per matrix pass (1, 2, 4, 8, 16, or 32 for 16-bit matrices; default 16)")
    ap.add_argument("--arith", type=int, default=0,
                    help="1: FP16 arithmetic for the FP16 matrices (the paper's half-precision variant)")
    ap.add_argument("--streamed", type=int, default=0, metavar="BATCH",
                    help="also time a step over BATCH host-resident slices (streamed entry points, chunks of "
                         "fuse slices, PCIe-inclusive)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (reference for profiler byte counters)")
    ap.add_argument("--dtype", default="f32", choices=["f32", "f16", "bf16", "f64"],
                    help="matrix/operand storage of the timed projection step (FP32 is the headline path; "
                         "f64 times FP64 slices, without CGLS)")
    args = ap.parse_args()

    if args.dtype == "f64":  # the FP64 variant: products only (CGLS runs on FP32 / 16-bit matrices)
        args.no_cgls = args.no_large = True
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

    oracle = None
    if not args.no_cpu:
        import oracle  # the CPU oracle leg only: timing and error reports
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))  # the host's oracle threads

    N, M, C, B = args.n, args.angles, args.n, args.batch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    default_opts = not (args.stage_order or args.lds_bytes or args.tile_waves or args.fuse or args.arith or
                        args.lane_order or args.slab_order or args.xcd_remap)

    log(f"building {args.dtype} matrix N={N} M={M} C={C}")
    opts = dict(stage_order=args.stage_order, lds_bytes=args.lds_bytes, tile_waves=args.tile_waves, fuse=args.fuse,
                lane_order=args.lane_order, slab_order=args.slab_order, xcd_remap=args.xcd_remap)
    opts16 = dict(opts, arith=args.arith)  # FP16 arithmetic applies to FP16 matrices only
    A = xct.Matrix(N, M, C, args.dtype, **(opts16 if args.dtype == "f16" else opts))
    info = A.info()
    log(f"built in {info['build_seconds']:.2f} s: A nnz {info['A']['nnz']:,} padded {info['A']['padded']:,}; "
        f"A^T padded {info['AT']['padded']:,}")
    nnz = info["A"]["nnz"]
    x = phantoms.ellipsoid_phantom(N, B, 40, seed=2, device=dev)
    x = x.double() if args.dtype == "f64" else x.float()

    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nb} bytes read, {nb} bytes written")
        del src, dst

    log(f"timing {args.steps} steps")
    hs = time_products(xct, torch, A, x, args.steps, warmup=args.warmup)
    F, ms_step = hs["fuse"], hs["ms_per_step"]
    bytes_step = hs["bytes_step"]
    value = bytes_step / (ms_step * 1e-3) / 1e9
    log(f"step {ms_step:.3f} ms ({hs['wall_ms_per_step']:.3f} ms wall), {value:.1f} GB/s; "
        f"SpMM A {hs['launch_ms']['A']:.3f} ms, A^T {hs['launch_ms']['AT']:.3f} ms per launch")
    y = xct.project(A, x)

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
            "achieved": hs["kernel_GBps"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": hs["kernel_frac"],
            "traffic": measured_traffic(args.dtype, N, M, B, default_opts),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "avg_launch_ms": hs["avg_launch_ms"],
            "alg_bytes_per_launch": hs["alg_bytes_per_launch"],
            "launch_ms": hs["launch_ms"],
        },
    }

    if oracle is not None:
        log("oracle errors of the headline products")
        out["oracle_error"] = headline_errors(oracle, xct, torch, A, N, M, C, x, y, [0, 7, 15])

    if args.streamed:
        # host-resident batch (the benchmark batch repeated): chunks of F slices
        # copied in and out on two copy streams while the SpMM runs;
        # PCIe-inclusive, never the headline value
        BS = args.streamed
        log(f"streamed step ({BS} host-resident slices)")
        b_a = BYTES_A[args.dtype]
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

        def cgls_history(Am):
            # untimed run with the per-iteration residual history ||y - A x_k|| / ||y||
            xo, res, _ = xct.cgls(Am, yc, it)
            return xo, res

        checkpoints = [k for k in (0, 1, 2, 3, 5, 10, 20, 30, 50) if k <= it]
        log("CGLS FP32")
        A32 = A if args.dtype == "f32" else xct.Matrix(N, M, C, "f32", **opts)
        t32 = cgls_s_per_iter(xct, torch, A32, yc, it)
        x32, res32 = cgls_history(A32)
        A32.free()
        A.free()
        del A32, A
        torch.cuda.empty_cache()
        log("building FP16 matrix")
        A16 = xct.Matrix(N, M, C, "f16", **opts16)
        log("CGLS FP16 storage")
        t16 = cgls_s_per_iter(xct, torch, A16, yc, it)
        x16, res16 = cgls_history(A16)
        d16 = ((x16 - x32).flatten(1).norm(dim=1) / x32.flatten(1).norm(dim=1).clamp_min(1e-30)).max().item()
        del x32, x16
        # the FP16 operators' projection + backprojection step, for reference
        s16 = time_products(xct, torch, A16, x, args.steps)
        out["fp16_step"] = {k: s16[k] for k in ("ms_per_step", "GBps", "kernel_GBps", "kernel_frac", "launch_ms",
                                                 "padded_A", "padded_AT")}
        if oracle is not None:
            out["fp16_step"]["oracle_error"] = product_errors(oracle, xct, torch, A16, x, [0, 15])
        # convergence against time: median relative residual over the slices
        # after k iterations, reached at k * s/iter
        out["cgls"] = {"iters": it, "fp32_s_per_iter": round(t32, 6), "fp16_s_per_iter": round(t16, 6),
                       "fp16_speedup": round(t32 / t16, 3),
                       "residual_median": {"k": checkpoints,
                                           "fp32": [float(np.median(res32[k])) for k in checkpoints],
                                           "fp16": [float(np.median(res16[k])) for k in checkpoints]},
                       "fp16_vs_fp32_rel_l2_max": round(d16, 6),
                       "build_s_f16": s16["build_s"]}
        log(f"CGLS s/iter FP32 {t32 * 1e3:.3f} ms, FP16 {t16 * 1e3:.3f} ms")
        # the gradient solver of Eq. (1) (x >= 0, TV) on the same FP16 operators
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
                                     "vs_spmm_pair": round(tpg / (s16["ms_per_step"] * 1e-3), 3)}
        A16.free()
        del A16
        # the paper's precision comparison (Sec. IV, CG time and convergence by
        # precision): CGLS with an FP64 matrix (FP64 vectors and sums) and with
        # FP16 arithmetic (FP16 matrix, packed FP16 sums), beside FP32 and mixed
        prec = {}
        for name, vdt, bopts in (("fp64", "f64", opts), ("half", "f16", dict(opts, arith=1))):
            log(f"CGLS {name}")
            Ap = xct.Matrix(N, M, C, vdt, **bopts)
            tp = cgls_s_per_iter(xct, torch, Ap, yc, it)
            _, resp = cgls_history(Ap)
            prec[name] = {"s_per_iter": round(tp, 6),
                          "residual_median": [float(np.median(resp[k])) for k in checkpoints]}
            Ap.free()
            del Ap
        out["cgls"]["precision"] = dict(prec, k=checkpoints,
                                        note="mixed = FP16 storage with FP32 sums (fp16 above); half = packed "
                                             "FP16 sums; fp64 = FP64 matrix, vectors and sums")
        del yc
    else:
        A.free()
        del A
    del y
    torch.cuda.empty_cache()

    traced = None
    if not args.no_large:
        # 64 slices 2048^2, 1500 angles, 2048 channels (FP32, FP16, BF16)
        N4, M4, B4, it4 = 2048, 1500, 64, 30
        sl4 = [17, 40]
        log("64 x 2048^2 x 1500: FP32 matrix")
        x4 = phantoms.ellipsoid_phantom(N4, B4, 60, seed=4, device=dev).float()
        c4 = {"workload": f"{B4} slices {N4}x{N4}, {M4} angles over [0,pi), {N4} channels, 60-ellipsoid phantom, "
                          f"1% noise; CGLS {it4} iterations"}
        if oracle is not None:
            # the oracle's CGLS history on 2 slices, on the host meanwhile
            x2 = x4[sl4].double().cpu().numpy().reshape(len(sl4), -1)
            traced = TracedOracleCgls(oracle, phantoms, N4, M4, N4, x2, sl4, 4, 3, max(1, threads - 2))
            traced.start()
            del x2
        y4 = y2 = None
        for dt in ("f32", "f16", "bf16"):
            A4 = xct.Matrix(N4, M4, N4, dt)
            if y4 is None:
                y4 = xct.project(A4, x4)
                y4 = (y4 + 0.01 * float(y4.abs().max()) * phantoms.noise_torch((M4, N4), B4, 4, dev)).contiguous()
            r = time_products(xct, torch, A4, x4, 3, warmup=1)
            if oracle is not None:
                r["oracle_error"] = product_errors(oracle, xct, torch, A4, x4, sl4)
            r["cgls_s_per_iter"] = round(cgls_s_per_iter(xct, torch, A4, y4, it4), 6)
            _, res4, _ = xct.cgls(A4, y4, it4)
            r["residual_median_final"] = float(np.median(res4[-1]))
            if traced is not None:
                if y2 is None and traced.sinogram() is not None:
                    y2 = torch.from_numpy(traced.sinogram()).float().reshape(len(sl4), M4, N4).to(dev)
                if y2 is not None:
                    r["_iterates"] = gpu_cgls_iterates(xct, A4, y2, 3)
            c4[dt] = r
            log(f"  {dt}: step {r['ms_per_step']:.2f} ms, kernel {100 * r['kernel_frac']:.1f}% of peak, "
                f"CGLS {1e3 * r['cgls_s_per_iter']:.2f} ms/iter")
            A4.free()
            del A4
            torch.cuda.empty_cache()
        # FP16 with 32 slices per matrix pass: half the matrix passes of the batch
        A4 = xct.Matrix(N4, M4, N4, "f16", fuse=32)
        r = time_products(xct, torch, A4, x4, 3, warmup=1)
        if oracle is not None:
            r["oracle_error"] = product_errors(oracle, xct, torch, A4, x4, sl4)
        r["cgls_s_per_iter"] = round(cgls_s_per_iter(xct, torch, A4, y4, it4), 6)
        c4["f16_fuse32"] = r
        log(f"  f16, 32 fused slices: step {r['ms_per_step']:.2f} ms, kernel {100 * r['kernel_frac']:.1f}% of peak, "
            f"CGLS {1e3 * r['cgls_s_per_iter']:.2f} ms/iter")
        A4.free()
        del A4
        torch.cuda.empty_cache()
        c4["fp16_cgls_speedup"] = round(c4["f32"]["cgls_s_per_iter"] / c4["f16"]["cgls_s_per_iter"], 3)
        c4["fp16_fuse32_cgls_speedup"] = round(c4["f32"]["cgls_s_per_iter"] / c4["f16_fuse32"]["cgls_s_per_iter"], 3)
        out["c64x2048"] = c4
        del x4, y4, y2
        torch.cuda.empty_cache()

        # 128 slices 2816^2, 2250 angles, 2816 channels, FP16 (the large single-GPU share)
        N5, M5, B5, it5 = 2816, 2250, 128, 20
        log("128 x 2816^2 x 2250: FP16 matrix")
        A5 = xct.Matrix(N5, M5, N5, "f16")
        x5 = phantoms.ellipsoid_phantom(N5, B5, 200, seed=5, device=dev, texture=0.05).float()
        r = time_products(xct, torch, A5, x5, 2, warmup=1)
        if oracle is not None:
            r["oracle_error"] = product_errors(oracle, xct, torch, A5, x5, [3, 100])
        y5 = xct.project(A5, x5)
        y5 = (y5 + 0.01 * float(y5.abs().max()) * phantoms.noise_torch((M5, N5), B5, 5, dev)).contiguous()
        del x5
        r["cgls_20_s"] = round(cgls_seconds(xct, torch, A5, y5, it5, reps=1), 4)
        r["cgls_s_per_iter"] = round((r["cgls_20_s"] - cgls_seconds(xct, torch, A5, y5, 0, reps=1)) / it5, 6)
        log(f"  f16: step {r['ms_per_step']:.2f} ms, kernel {100 * r['kernel_frac']:.1f}% of peak, "
            f"{it5} CGLS iterations {r['cgls_20_s']:.2f} s")
        out["c128x2816"] = {"workload": f"{B5} slices {N5}x{N5}, {M5} angles over [0,pi), {N5} channels, "
                                        f"200 ellipsoids + texture, 1% noise; CGLS {it5} iterations", "f16": r}
        A5.free()
        del A5
        torch.cuda.empty_cache()
        A5 = xct.Matrix(N5, M5, N5, "f16", fuse=32)
        x5 = phantoms.ellipsoid_phantom(N5, B5, 200, seed=5, device=dev, texture=0.05).float()
        r = time_products(xct, torch, A5, x5, 2, warmup=1)
        if oracle is not None:
            r["oracle_error"] = product_errors(oracle, xct, torch, A5, x5, [3, 100])
        del x5
        r["cgls_20_s"] = round(cgls_seconds(xct, torch, A5, y5, it5, reps=1), 4)
        r["cgls_s_per_iter"] = round((r["cgls_20_s"] - cgls_seconds(xct, torch, A5, y5, 0, reps=1)) / it5, 6)
        log(f"  f16, 32 fused slices: step {r['ms_per_step']:.2f} ms, kernel {100 * r['kernel_frac']:.1f}% of "
            f"peak, {it5} CGLS iterations {r['cgls_20_s']:.2f} s")
        out["c128x2816"]["f16_fuse32"] = r
        A5.free()
        del A5, y5
        torch.cuda.empty_cache()

    if oracle is not None:
        oracle.set_threads(threads)
        log("CGLS against the oracle per iteration, 2 slices of 512^2 x 360")
        out["cgls_vs_oracle_512"] = cgls_errors_512(oracle, xct, torch, phantoms, dev)
        if traced is not None:
            log("waiting for the oracle's 2048^2 CGLS")
            traced.join()
            oracle.set_threads(threads)
            c4 = out["c64x2048"]
            rep = {"slices": sl4, "k": [1, 2, 3], "oracle_seconds": round(traced.seconds, 1)}
            if traced.result is not None and all("_iterates" in c4[dt] for dt in ("f32", "f16", "bf16")):
                xho, reso = traced.result
                for dt in ("f32", "f16", "bf16"):
                    xg, resg = c4[dt].pop("_iterates")
                    rep[dt] = [round(e, 8) for e in per_iteration_errors(xg, xho)]
                    rep[dt + "_residual_rel_dev_max"] = float((abs(resg - reso) / reso).max())
                rep["f16_within_1e-3_through_k"] = holds_through(rep["f16"], 1e-3)
            else:
                rep["error"] = traced.error or "no GPU iterates"
                for dt in ("f32", "f16", "bf16"):
                    c4[dt].pop("_iterates", None)
            c4["cgls_vs_oracle"] = rep
        log("CPU oracle baseline")
        ys = np.random.default_rng(1).random((B, M * C))
        out["cpu_baseline"] = cpu_baseline(oracle, N, M, C, B, x.double().cpu().numpy().reshape(B, -1), ys,
                                           bytes_step, args.cpu_seconds, threads)
    elif "c64x2048" in out:
        for dt in ("f32", "f16", "bf16"):
            out["c64x2048"][dt].pop("_iterates", None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
