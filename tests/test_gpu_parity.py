"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bars: FP32 projection / backprojection within 1e-5 relative L2 per slice of
the oracle on phantom inputs (the target fixed for the plain path); matrix
entries equal to the oracle's FP64 lengths rounded once to the stored dtype
(1 ulp allowed for the last-bit differences of device vs host sin/cos);
CGLS against the oracle's history at every iteration up to the fixed count:
within 1e-5 over the first iterations, and within twice the rounding
envelope of the kernel's arithmetic (tests/cgls_envelope.py) at every k,
with FP32 held to 1e-4 and FP16 storage to 1e-3 at every k where that
envelope admits it (the envelope grows about tenfold per iteration once
rounding is amplified, so no non-FP64 solver matches FP64 iterates tightly
past that point).
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2009_07226_amd import phantoms

pytestmark = pytest.mark.gpu

xct = pytest.importorskip("paper_2009_07226_amd")

_cache = {}


def gpu_matrix(N, M, C, dt="f32", **kw):
    key = (N, M, C, dt, tuple(sorted(kw.items())))
    if key not in _cache:
        _cache[key] = xct.Matrix(N, M, C, dt, **kw)
    return _cache[key]


def oracle_mats(N, M, C):
    key = ("oracle", N, M, C)
    if key not in _cache:
        _cache[key] = (oracle.build_A(N, M, C), oracle.build_AT(N, M, C))
    return _cache[key]


def rel_err(a, b):
    a = np.asarray(a, np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, np.float64).reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


GEOMS = [(128, 180, 128), (37, 23, 41), (16, 12, 16), (24, 10, 23), (5, 7, 6), (64, 1, 64)]


@pytest.mark.parametrize("N,M,C", GEOMS)
@pytest.mark.parametrize("dt", ["f32", "f16", "bf16"])
def test_matrix_entries_match_oracle(N, M, C, dt):
    banner(f"entries N={N} M={M} C={C} {dt}")
    A = gpu_matrix(N, M, C, dt)
    Ao, ATo = oracle_mats(N, M, C)
    npdt = {"f32": np.float32, "f16": np.float16, "bf16": None}[dt]
    for which, ref in ((0, Ao.tocoo()), (1, ATo.tocoo())):
        r, c, v = A.to_coo(which)
        if dt == "bf16":
            rv = torch.from_numpy(ref.data).to(torch.bfloat16).float().numpy()
        else:
            rv = ref.data.astype(npdt).astype(np.float32)
        keep = rv != 0
        rk = ref.row[keep].astype(np.int64) * ref.shape[1] + ref.col[keep]
        gk = r.astype(np.int64) * ref.shape[1] + c
        assert len(np.unique(gk)) == len(gk), "duplicate entries"
        og, oo = np.argsort(gk), np.argsort(rk)
        np.testing.assert_array_equal(gk[og], rk[oo])
        gv, ov = v[og], rv[keep][oo]
        if dt == "f32":
            ulp = np.spacing(ov.astype(np.float32))
        elif dt == "f16":
            ulp = np.spacing(ov.astype(np.float16)).astype(np.float32)
        else:
            ulp = np.abs(ov) * 2.0 ** -7
        assert np.all(np.abs(gv - ov) <= ulp), np.abs(gv - ov).max()
        # lengths that round to zero in the stored format are not entries
        info = A.info()["AT" if which else "A"]
        assert info["nnz"] == int(keep.sum())


@pytest.mark.parametrize("dt", ["f32", "f16"])
@pytest.mark.parametrize("N,M,C", [(128, 180, 128), (37, 23, 41)])
def test_matrix_entries_two_row_tiles_per_wavefront(N, M, C, dt):
    # 32 row tiles per block on 16 wavefronts: every entry decodes to the
    # oracle's (row, column) once, with its rounded length
    banner(f"entries W=32 N={N} M={M} C={C} {dt}")
    A = gpu_matrix(N, M, C, dt, tile_waves=32)
    Ao, ATo = oracle_mats(N, M, C)
    npdt = {"f32": np.float32, "f16": np.float16}[dt]
    for which, ref in ((0, Ao.tocoo()), (1, ATo.tocoo())):
        r, c, v = A.to_coo(which)
        rv = ref.data.astype(npdt).astype(np.float32)
        keep = rv != 0
        rk = ref.row[keep].astype(np.int64) * ref.shape[1] + ref.col[keep]
        gk = r.astype(np.int64) * ref.shape[1] + c
        og, oo = np.argsort(gk), np.argsort(rk)
        np.testing.assert_array_equal(gk[og], rk[oo])
        gv, ov = v[og], rv[keep][oo]
        ulp = np.spacing(ov.astype(npdt)).astype(np.float32)
        assert np.all(np.abs(gv - ov) <= ulp), np.abs(gv - ov).max()


@pytest.mark.parametrize("N,M,C", GEOMS)
@pytest.mark.parametrize("B", [1, 3, 16, 17])
def test_project_backproject_parity(N, M, C, B):
    banner(f"spmm N={N} M={M} C={C} B={B}")
    A = gpu_matrix(N, M, C)
    Ao, ATo = oracle_mats(N, M, C)
    x = phantoms.ellipse_batch(N, B, 6, seed=100 + B).float()
    y_gpu = xct.project(A, x.cuda()).cpu()
    y_ref = oracle.project(Ao, x.double().numpy().reshape(B, -1))
    e = rel_err(y_gpu.numpy(), y_ref)
    assert e.max() <= 1e-5, e
    yin = (torch.from_numpy(y_ref).float() + 0.1 * torch.randn(B, M * C, generator=torch.Generator().manual_seed(B)))
    yin = yin.reshape(B, M, C)
    xb_gpu = xct.backproject(A, yin.cuda()).cpu()
    xb_ref = oracle.backproject(ATo, yin.double().numpy())
    e = rel_err(xb_gpu.numpy(), xb_ref)
    assert e.max() <= 1e-5, e


@pytest.mark.parametrize("opts", [dict(stage_order=1), dict(tile_waves=4, lds_bytes=32768),
                                  dict(tile_waves=16, xcd_remap=-1), dict(xcd_remap=1), dict(xcd_remap=3),
                                  dict(tile_waves=5, xcd_remap=7), dict(fuse=4), dict(fuse=2),
                                  dict(lane_order=1), dict(tile_waves=16, lds_bytes=163840),
                                  dict(slab_order=1), dict(fuse=8), dict(fuse=8, lane_order=1),
                                  dict(tile_waves=32), dict(tile_waves=32, fuse=8), dict(tile_waves=32, fuse=1),
                                  dict(tile_waves=32, fuse=4, lds_bytes=32768), dict(tile_waves=32, slab_order=1)])
def test_plan_options_keep_parity(opts):
    N, M, C, B = 64, 90, 64, 5
    A = gpu_matrix(N, M, C, **opts)
    Ao, ATo = oracle_mats(N, M, C)
    x = phantoms.ellipse_batch(N, B, 6, seed=21).float()
    y_ref = oracle.project(Ao, x.double().numpy().reshape(B, -1))
    y = xct.project(A, x.cuda()).cpu()
    assert rel_err(y.numpy(), y_ref).max() <= 1e-5
    yin = torch.from_numpy(y_ref).float().reshape(B, M, C)  # the oracle's sinogram, as FP32 input
    xb = xct.backproject(A, yin.cuda()).cpu()
    assert rel_err(xb.numpy(), oracle.backproject(ATo, yin.double().numpy())).max() <= 1e-5


@pytest.mark.parametrize("dt,tol", [("f16", 2e-3), ("bf16", 1.5e-2)])
@pytest.mark.parametrize("opts", [dict(lane_order=1), dict(tile_waves=32), dict(tile_waves=5, xcd_remap=7),
                                  dict(fuse=1), dict(fuse=2), dict(fuse=8, lane_order=1), dict(stage_order=1),
                                  dict(slab_order=1), dict(tile_waves=4, lds_bytes=16384)])
def test_plan_options_keep_parity_16bit(opts, dt, tol):
    # 16-bit matrices write their sums straight into the natural output (the
    # product's epilogue maps each lane's row to its pixel): every lane order,
    # row tiles per wavefront, block order and fused slice count, with 16-bit
    # and FP32 io, within the storage-rounding bars
    N, M, C, B = 64, 90, 64, 5
    A = gpu_matrix(N, M, C, dt, **opts)
    Ao, ATo = oracle_mats(N, M, C)
    x = phantoms.ellipse_batch(N, B, 6, seed=23).float()
    y_ref = oracle.project(Ao, x.double().numpy().reshape(B, -1))
    yin = torch.from_numpy(y_ref).float().reshape(B, M, C)  # the oracle's sinogram, as input
    xb_ref = oracle.backproject(ATo, yin.double().numpy())
    io16 = torch.float16 if dt == "f16" else torch.bfloat16
    for io in (torch.float32, io16):
        y = xct.project(A, x.to(io).cuda())
        assert y.dtype == io
        e = rel_err(y.float().cpu().numpy(), y_ref)
        xb = xct.backproject(A, yin.to(io).cuda())
        eb = rel_err(xb.float().cpu().numpy(), xb_ref)
        banner(f"{dt} {opts} io={io}: projection {e.max():.2e} backprojection {eb.max():.2e}")
        # 16-bit input and output each add their own rounding (at most half
        # an ulp: 2^-11 relative in FP16, 2^-8 in BF16)
        bar = tol if io == torch.float32 else tol + 2 * (2.0 ** -11 if dt == "f16" else 2.0 ** -8)
        assert e.max() <= bar and eb.max() <= bar


@pytest.mark.parametrize("dt,kw,expect", [("f32", {}, True), ("f16", {}, True), ("bf16", {}, True),
                                           ("f32", dict(fuse=8), True), ("f32", dict(slab_order=1), False),
                                           ("f32", dict(fuse=4), False), ("f16", dict(fuse=8), False)])
def test_slab_scheduling_applied(dt, kw, expect):
    # rows of 32 or 64 bytes get the bank-conflict schedule, every slab of it
    A = gpu_matrix(128, 180, 128, dt, **kw)
    for op in ("A", "AT"):
        st = A.info()[op]
        assert st["slabs"] > 0
        assert st["balanced_slabs"] == (st["slabs"] if expect else 0), st


def test_output_shape_and_zero_input():
    A = gpu_matrix(37, 23, 41)
    y = xct.project(A, torch.zeros(2, 37, 37, device="cuda"))
    assert y.shape == (2, 23, 41) and float(y.abs().max()) == 0.0
    x = xct.backproject(A, torch.zeros(2, 23, 41, device="cuda"))
    assert x.shape == (2, 37, 37) and float(x.abs().max()) == 0.0


def test_bitwise_deterministic_and_batch_independent():
    N, M, C = 128, 180, 128
    A = gpu_matrix(N, M, C)
    x = phantoms.ellipse_batch(N, 16, 8, seed=5).float().cuda()
    y1 = xct.project(A, x)
    y2 = xct.project(A, x)
    assert torch.equal(y1, y2)
    # one slice alone through a 1-slice pass agrees with the fused pass
    y3 = xct.project(A, x[5:6].contiguous())
    e = (y3[0] - y1[5]).norm() / y1[5].norm()
    assert float(e) <= 1e-6
    b1 = xct.backproject(A, y1)
    b2 = xct.backproject(A, y1)
    assert torch.equal(b1, b2)


def test_adjoint_identity_on_gpu():
    N, M, C = 128, 180, 128
    A = gpu_matrix(N, M, C)
    g = torch.Generator(device="cuda").manual_seed(3)
    x = torch.randn(4, N, N, device="cuda", generator=g)
    y = torch.randn(4, M, C, device="cuda", generator=g)
    Ax = xct.project(A, x).double()
    ATy = xct.backproject(A, y).double()
    lhs = (Ax * y.double()).sum(dim=(1, 2))
    rhs = (x.double() * ATy).sum(dim=(1, 2))
    scale = Ax.flatten(1).norm(dim=1) * y.double().flatten(1).norm(dim=1)
    assert float(((lhs - rhs).abs() / scale).max()) <= 1e-6


@pytest.mark.parametrize("dt,tol", [("f16", 2e-3), ("bf16", 1.5e-2)])
def test_reduced_precision_projection_error(dt, tol):
    N, M, C, B = 128, 180, 128, 4
    A = gpu_matrix(N, M, C, dt)
    Ao, ATo = oracle_mats(N, M, C)
    x = phantoms.ellipse_batch(N, B, 8, seed=9).float()
    y_ref = oracle.project(Ao, x.double().numpy().reshape(B, -1))
    for io in (torch.float32, torch.float16 if dt == "f16" else torch.bfloat16):
        y = xct.project(A, x.to(io).cuda()).float().cpu().numpy()
        e = rel_err(y, y_ref)
        banner(f"{dt} io={io} projection rel err {e.max():.2e}")
        assert e.max() <= tol
    yb = torch.from_numpy(y_ref.reshape(B, M, C)).float()
    xb = xct.backproject(A, yb.cuda()).cpu().numpy()
    e = rel_err(xb, oracle.backproject(ATo, yb.double().numpy()))
    banner(f"{dt} backprojection rel err {e.max():.2e}")
    assert e.max() <= tol


@pytest.mark.parametrize("dt,tol", [("f16", 2e-3), ("bf16", 1.5e-2)])
@pytest.mark.parametrize("N,M,C", [(128, 180, 128), (37, 23, 41)])
def test_fuse32_parity(dt, tol, N, M, C):
    # 32 slices per matrix pass (16-bit operands): ragged batches around one
    # and two full passes, both products, within the storage-rounding bars
    A = gpu_matrix(N, M, C, dt, fuse=32)
    assert A.info()["fuse"] == 32
    Ao, ATo = oracle_mats(N, M, C)
    for B in (1, 17, 32, 33, 70):
        x = phantoms.ellipse_batch(N, B, 5, seed=300 + B).float()
        y_ref = oracle.project(Ao, x.double().numpy().reshape(B, -1))
        y = xct.project(A, x.cuda())
        e = rel_err(y.cpu().numpy(), y_ref)
        yin = torch.from_numpy(y_ref).float().reshape(B, M, C)  # the oracle's sinogram, as FP32 input
        xb = xct.backproject(A, yin.cuda())
        eb = rel_err(xb.cpu().numpy(), oracle.backproject(ATo, yin.double().numpy()))
        banner(f"fuse 32 {dt} N={N} B={B}: projection {e.max():.2e} backprojection {eb.max():.2e}")
        assert e.max() <= tol and eb.max() <= tol


def test_fuse32_needs_16bit_matrix():
    with pytest.raises(xct.XctError) as e:
        xct.Matrix(16, 12, 16, "f32", fuse=32)
    assert e.value.code == -4
    with pytest.raises(xct.XctError) as e:
        xct.Matrix(16, 12, 16, "f16", fuse=32, tile_waves=32)
    assert e.value.code == -4


def test_cgls_fuse32_early_iterations():
    # FP16 storage with 32 fused slices: a 33-slice batch (a full pass and a
    # one-slice pass) within the 1e-3 gate of the oracle over 3 iterations
    N, M, C, B = 64, 90, 64, 33
    A = gpu_matrix(N, M, C, "f16", fuse=32)
    Ao, ATo, _, y = cgls_problem(N, M, C, B, seed=6)
    xg, resg, stg = xct.cgls(A, y.cuda(), 3)
    xo, reso, sto = oracle.cgls(Ao, ATo, y.double().numpy().reshape(B, -1), 3)
    e = rel_err(xg.cpu().numpy(), xo)
    banner(f"cgls fuse 32 f16 B={B} k=3 rel err {e.max():.2e}")
    assert e.max() <= 1e-3
    assert np.all(stg == sto)


def noisy_sinogram(Ao, x, sigma_frac, seed, M, C):
    y = oracle.project(Ao, x.double().numpy().reshape(x.shape[0], -1))
    sigma = sigma_frac * y.max()
    nz = phantoms.noise((M * C,), range(x.shape[0]), seed)
    return torch.from_numpy(y + sigma * nz).float().reshape(x.shape[0], M, C)


CGLS_CASES = [(128, 180, 128, 1, 10), (37, 23, 41, 5, 8), (64, 90, 64, 17, 12)]


def cgls_problem(N, M, C, B, seed=1):
    Ao, ATo = oracle_mats(N, M, C)
    x_true = phantoms.ellipse_batch(N, B, 10, seed=seed).float()
    return Ao, ATo, x_true, noisy_sinogram(Ao, x_true, 0.01, seed, M, C)


@pytest.mark.parametrize("N,M,C,B,iters", CGLS_CASES)
def test_cgls_early_iterations_match_oracle(N, M, C, B, iters):
    # Over the first iterations rounding has not yet been amplified by the
    # recurrences (see test_cgls_iterates_amplify_rounding): tight parity.
    banner(f"cgls early N={N} M={M} C={C} B={B}")
    A = gpu_matrix(N, M, C)
    Ao, ATo, _, y = cgls_problem(N, M, C, B)
    for k in (1, 2, 4):
        xg, resg, stg = xct.cgls(A, y.cuda(), k)
        xo, reso, sto = oracle.cgls(Ao, ATo, y.double().numpy().reshape(B, -1), k)
        e = rel_err(xg.cpu().numpy(), xo)
        banner(f"  k={k} rel err {e.max():.2e}")
        assert e.max() <= 1e-5, e
        np.testing.assert_allclose(resg, reso, rtol=1e-5, atol=1e-8)
        assert np.all(stg == sto)


def test_cgls_two_row_tiles_per_wavefront():
    # the per-block sums of squares cover both row tiles of each wavefront
    N, M, C, B = 64, 90, 64, 5
    A = gpu_matrix(N, M, C, tile_waves=32)
    Ao, ATo, _, y = cgls_problem(N, M, C, B)
    for k in (1, 4):
        xg, resg, stg = xct.cgls(A, y.cuda(), k)
        xo, reso, sto = oracle.cgls(Ao, ATo, y.double().numpy().reshape(B, -1), k)
        assert rel_err(xg.cpu().numpy(), xo).max() <= 1e-5
        np.testing.assert_allclose(resg, reso, rtol=1e-5, atol=1e-8)
        assert np.all(stg == sto)


def gpu_cgls_history(A, y, iters):
    """x_1..x_iters of the GPU CGLS as (iters, B, cols) FP64, one run per k
    (the solver is deterministic, so a k-iteration run returns the k-th
    iterate of any longer run), and the residual history and status of the
    iters-iteration run."""
    B = y.shape[0]
    xs = []
    for k in range(1, iters + 1):
        x, res, st = xct.cgls(A, y, k)
        xs.append(x.double().cpu().numpy().reshape(B, -1))
    return np.stack(xs), res, st


def check_cgls_history(xg, resg, xo, reso, env_x, env_r, label, gate=None):
    """Per-iteration bars against the oracle's history: the iterate within
    2x the rounding envelope of its storage format, the residual norm within
    2x its envelope plus the FP32 rounding of the stored residual (2 u32
    relative to ||y||, i.e. 2 u32 / r_k relative to r_k).  ``gate``: also
    require ||x_k - x_k*|| / ||x_k*|| <= gate at every k where the envelope
    allows it (2 env_x <= gate).  Returns (dev_x, dev_r), (iters+1, B), and
    the last k at which the measured deviation is within ``gate``."""
    iters = xg.shape[0]
    dev_x = np.zeros_like(env_x)
    for k in range(1, iters + 1):
        dev_x[k] = rel_err(xg[k - 1], xo[k - 1])
    dev_r = np.abs(resg - reso) / np.maximum(reso, 1e-300)
    floor_r = 2 * 2.0 ** -24 / np.maximum(reso, 1e-300)
    for k in range(1, iters + 1):
        banner(f"  {label} k={k:2d} x dev {dev_x[k].max():.2e} (envelope {env_x[k].max():.2e})  "
               f"resid dev {dev_r[k].max():.2e} (envelope {env_r[k].max():.2e})")
    assert np.all(dev_x <= 2 * env_x), (label, dev_x.max(axis=1), env_x.max(axis=1))
    assert np.all(dev_r <= 2 * env_r + floor_r), (label, dev_r.max(axis=1), env_r.max(axis=1))
    k_gate = None
    if gate is not None:
        within = [k for k in range(1, iters + 1) if dev_x[k].max() <= gate]
        k_gate = max([0] + [k for k in range(1, iters + 1) if all(dev_x[j].max() <= gate for j in range(1, k + 1))])
        enforced = [k for k in range(1, iters + 1) if 2 * env_x[k].max() <= gate]
        banner(f"  {label}: {gate:g} gate enforced for k in {enforced}, holds through k={k_gate} "
               f"(and at k in {within})")
        for k in enforced:
            assert dev_x[k].max() <= gate, (label, k, dev_x[k])
    return dev_x, dev_r, k_gate


@pytest.mark.parametrize("N,M,C,B,iters", CGLS_CASES)
def test_cgls_every_iteration_within_rounding_envelope(N, M, C, B, iters):
    """FP32 CGLS against the oracle at every iteration up to the fixed count:
    iterates and residual norms within 2x the FP32 rounding envelope (the
    largest deviation of 16 FP32 solvers that sum in other orders), and
    within 1e-4 relative L2 of the oracle wherever the envelope admits it."""
    from cgls_envelope import envelope_history
    banner(f"cgls per iteration N={N} M={M} C={C} B={B} iters={iters}")
    A = gpu_matrix(N, M, C)
    Ao, ATo, x_true, y = cgls_problem(N, M, C, B)
    yd = y.double().numpy().reshape(B, -1)
    xg, resg, stg = gpu_cgls_history(A, y.cuda(), iters)
    xo, reso, sto, xho = oracle.cgls(Ao, ATo, yd, iters, history=True)
    env_x, env_r = envelope_history(Ao, ATo, yd, xho, reso, iters, storage="f32", seeds=tuple(range(16)))
    check_cgls_history(xg, resg, xho, reso, env_x, env_r, "f32", gate=1e-4)
    assert np.all(stg == sto)
    # the reconstruction is as good as the oracle's against the phantom
    xt = x_true.double().numpy().reshape(B, -1)
    assert np.all(rel_err(xg[-1], xt) <= 1.2 * rel_err(xo, xt))


def test_cgls_zero_sinogram_slice_stops():
    N, M, C, B = 37, 23, 41, 3
    A = gpu_matrix(N, M, C)
    Ao, _ = oracle_mats(N, M, C)
    y = noisy_sinogram(Ao, phantoms.ellipse_batch(N, B, 5, seed=2).float(), 0.01, 2, M, C)
    y[1] = 0
    x, res, st = xct.cgls(A, y.cuda(), 6)
    assert st[1] == 1 and st[0] == 0 and st[2] == 0
    assert float(x[1].abs().max()) == 0.0 and np.all(res[:, 1] == 0.0)


def test_cgls_zero_iterations():
    N, M, C = 16, 12, 16
    A = gpu_matrix(N, M, C)
    y = torch.rand(2, M, C, device="cuda")
    x, res, st = xct.cgls(A, y, 0)
    assert float(x.abs().max()) == 0.0 and np.all(res[0] == 1.0)


@pytest.mark.parametrize("dt", ["f16", "bf16"])
def test_cgls_reduced_precision_every_iteration_512(dt):
    """16-bit storage (matrix values and SpMM operands; FP32 sums, FP64
    scalars) against the FP64 oracle on 2 slices of 512^2, 360 angles, 512
    channels, 1% noise, at every one of 30 iterations: iterates and residual
    norms within 2x the rounding envelope of the storage format (3 solvers
    that round the same data to 16 bits and sum in other orders), and for
    FP16 the 1e-3 gate wherever that envelope admits it."""
    from cgls_envelope import envelope_history
    N, M, C, B, iters = 512, 360, 512, 2, 30
    banner(f"cgls {dt} per iteration N={N} M={M} B={B} iters={iters}")
    A16 = gpu_matrix(N, M, C, dt)
    Ao, ATo = oracle_mats(N, M, C)
    x_true = phantoms.ellipsoid_phantom(N, 8, 20, seed=3)[[2, 5]].float()
    y = noisy_sinogram(Ao, x_true, 0.01, 3, M, C)
    yd = y.double().numpy().reshape(B, -1)
    xg, resg, stg = gpu_cgls_history(A16, y.cuda(), iters)
    xo, reso, sto, xho = oracle.cgls(Ao, ATo, yd, iters, history=True)
    env_x, env_r = envelope_history(Ao, ATo, yd, xho, reso, iters, storage=dt)
    check_cgls_history(xg, resg, xho, reso, env_x, env_r, dt, gate=1e-3 if dt == "f16" else None)
    assert np.all(stg == sto)
    xt = x_true.double().numpy().reshape(B, -1)
    assert np.all(rel_err(xg[-1], xt) <= 1.2 * rel_err(xo, xt))


def test_autograd_pair_matches_oracle_and_finite_differences():
    N, M, C, B = 64, 90, 64, 2
    A = gpu_matrix(N, M, C)
    Ao, ATo = oracle_mats(N, M, C)
    x_true = phantoms.ellipse_batch(N, B, 6, seed=7).float()
    y = noisy_sinogram(Ao, x_true, 0.02, 7, M, C)
    x0 = (0.5 * x_true).cuda().requires_grad_(True)
    loss = 0.5 * ((xct.XctProject.apply(x0, A) - y.cuda()) ** 2).sum()
    loss.backward()
    g = x0.grad.double().cpu().numpy().reshape(B, -1)
    xd = x0.detach().double().cpu().numpy().reshape(B, -1)
    r = oracle.project(Ao, xd) - y.double().numpy().reshape(B, -1)
    g_ref = oracle.backproject(ATo, r)
    assert rel_err(g, g_ref).max() <= 1e-5
    # central differences of the FP64 loss on 64 seeded voxels, h = 1e-3
    rng = np.random.default_rng(0)
    idx = rng.choice(N * N, 64, replace=False)
    h = 1e-3
    for b in range(B):
        fd = []
        for v in idx:
            xp, xm = xd[b].copy(), xd[b].copy()
            xp[v] += h
            xm[v] -= h
            lp = 0.5 * np.sum((oracle.project(Ao, xp[None])[0] - y[b].double().numpy().ravel()) ** 2)
            lm = 0.5 * np.sum((oracle.project(Ao, xm[None])[0] - y[b].double().numpy().ravel()) ** 2)
            fd.append((lp - lm) / (2 * h))
        fd = np.array(fd)
        assert np.linalg.norm(g[b, idx] - fd) <= 1e-4 * np.linalg.norm(fd)
    # backprojection's backward is the projection
    yv = y.cuda().requires_grad_(True)
    out = xct.XctBackproject.apply(yv, A)
    w = torch.randn_like(out)
    (out * w).sum().backward()
    ref = xct.project(A, w)
    assert float((yv.grad - ref).abs().max()) == 0.0


def test_sampled_rows_at_size_512():
    # 8 slices of 512^2, 360 angles, 512 channels: sampled rows and voxels
    # against the oracle traced one by one (the full CSR would be 1.4 GB).
    N, M, C, B = 512, 360, 512, 8
    banner("sampled parity N=512")
    A = gpu_matrix(N, M, C)
    x = phantoms.ellipsoid_phantom(N, B, 20, seed=3).float()
    y = xct.project(A, x.cuda()).cpu()
    rng = np.random.default_rng(11)
    rows = rng.choice(M * C, 400, replace=False)
    ref = oracle.project_rows(N, M, C, x.double().numpy(), rows)
    got = y.reshape(B, -1)[:, rows].double().numpy()
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()
    vox = rng.choice(N * N, 400, replace=False)
    ys = torch.rand(B, M, C, generator=torch.Generator().manual_seed(12))
    xb = xct.backproject(A, ys.cuda()).cpu()
    ref = oracle.backproject_voxels(N, M, C, ys.double().numpy(), vox)
    got = xb.reshape(B, -1)[:, vox].double().numpy()
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("B", [5, 16])
def test_fp16_arithmetic_within_rounding_bound(B):
    # The paper's "half precision" variant: FP16 storage and FP16 sums.  Each
    # of a row's k additions rounds to 11 bits; with round-to-nearest the
    # errors behave like a random walk, so the relative error of a sum stays
    # within a few sqrt(k) * 2^-11 (here 4x, plus the operand's own rounding).
    N, M, C = 128, 180, 128
    Ao, ATo = oracle_mats(N, M, C)
    A16 = gpu_matrix(N, M, C, "f16")
    A16h = gpu_matrix(N, M, C, "f16", arith=1)
    x = phantoms.ellipse_batch(N, B, 6, seed=31).float()
    xr = oracle.project(Ao, x.double().numpy().reshape(B, -1))
    u = 2.0 ** -11
    bound_A = 4 * np.sqrt(Ao.getnnz(axis=1).max()) * u + 2 * u
    y16 = xct.project(A16, x.cuda()).cpu()
    y16h = xct.project(A16h, x.cuda()).cpu()
    e = rel_err(y16h.numpy(), xr)
    banner(f"FP16 arithmetic A x: max rel err {e.max():.2e} (bound {bound_A:.2e}); FP32 sums "
           f"{rel_err(y16.numpy(), xr).max():.2e}")
    assert e.max() <= bound_A
    assert not torch.equal(y16h, y16)  # the FP16-sum kernel ran
    yr = torch.from_numpy(xr).float().reshape(B, M, C)
    xb = xct.backproject(A16h, yr.cuda()).cpu()
    bound_AT = 4 * np.sqrt(ATo.getnnz(axis=1).max()) * u + 2 * u
    e = rel_err(xb.numpy(), oracle.backproject(ATo, yr.double().numpy()))
    assert e.max() <= bound_AT


def test_fp16_arithmetic_options():
    with pytest.raises(xct.XctError):
        gpu_matrix(16, 12, 16, "f32", arith=1)
    with pytest.raises(xct.XctError):
        gpu_matrix(16, 12, 16, "bf16", arith=1)
    # a single fused slice keeps FP32 sums
    A16 = gpu_matrix(37, 23, 41, "f16")
    A16h = gpu_matrix(37, 23, 41, "f16", arith=1)
    x = phantoms.ellipse_batch(37, 1, 4, seed=5).float().cuda()
    assert torch.equal(xct.project(A16, x), xct.project(A16h, x))


# ---- FP64 matrices (the double-precision variant) -------------------------------

@pytest.mark.parametrize("N,M,C", GEOMS)
def test_fp64_products_match_oracle(N, M, C):
    # FP64 lengths, operands and sums: within 1e-12 of the oracle per slice,
    # ragged batches around the 8-slice pass
    A = gpu_matrix(N, M, C, "f64")
    info = A.info()
    assert info["fuse"] == 8 and info["A"]["nnz"] == oracle_mats(N, M, C)[0].nnz
    Ao, ATo = oracle_mats(N, M, C)
    for B in (1, 8, 9):
        x = phantoms.ellipse_batch(N, B, 6, seed=500 + B).double()
        y = xct.project(A, x.cuda())
        assert y.dtype == torch.float64
        e = rel_err(y.cpu().numpy(), oracle.project(Ao, x.numpy().reshape(B, -1)))
        yin = torch.from_numpy(oracle.project(Ao, x.numpy().reshape(B, -1))).reshape(B, M, C)
        yin = yin + 0.1 * torch.randn(B, M, C, generator=torch.Generator().manual_seed(B), dtype=torch.float64)
        xb = xct.backproject(A, yin.cuda())
        eb = rel_err(xb.cpu().numpy(), oracle.backproject(ATo, yin.numpy()))
        banner(f"f64 N={N} M={M} C={C} B={B}: projection {e.max():.2e} backprojection {eb.max():.2e}")
        assert e.max() <= 1e-12 and eb.max() <= 1e-12


def test_fp64_entries_and_io():
    N, M, C = 37, 23, 41
    A = gpu_matrix(N, M, C, "f64")
    Ao, ATo = oracle_mats(N, M, C)
    for which, ref in ((0, Ao.tocoo()), (1, ATo.tocoo())):
        r, c, v = A.to_coo(which)  # lengths decoded as FP32
        gk = r.astype(np.int64) * ref.shape[1] + c
        rk = ref.row.astype(np.int64) * ref.shape[1] + ref.col
        og, oo = np.argsort(gk), np.argsort(rk)
        np.testing.assert_array_equal(gk[og], rk[oo])
        ov = ref.data[oo].astype(np.float32)
        assert np.all(np.abs(v[og] - ov) <= np.spacing(ov))
    # FP32 io on an FP64 matrix: the operand rounded once, sums in FP64
    x = phantoms.ellipse_batch(N, 3, 5, seed=41).float()
    y = xct.project(A, x.cuda())
    assert y.dtype == torch.float32
    assert rel_err(y.cpu().numpy(), oracle.project(Ao, x.double().numpy().reshape(3, -1))).max() <= 1e-6
    # adjoint identity in FP64
    g = torch.Generator(device="cuda").manual_seed(5)
    xr = torch.randn(2, N, N, device="cuda", dtype=torch.float64, generator=g)
    yr = torch.randn(2, M, C, device="cuda", dtype=torch.float64, generator=g)
    lhs = (xct.project(A, xr) * yr).sum(dim=(1, 2))
    rhs = (xr * xct.backproject(A, yr)).sum(dim=(1, 2))
    assert float(((lhs - rhs).abs() / lhs.abs().clamp_min(1e-300)).max()) <= 1e-12


def test_fp64_limits():
    with pytest.raises(xct.XctError) as e:
        xct.Matrix(16, 12, 16, "f64", fuse=16)
    assert e.value.code == -4


@pytest.mark.parametrize("N,M,C,B,iters", CGLS_CASES)
def test_fp64_cgls_every_iteration(N, M, C, B, iters):
    """CGLS on an FP64 matrix (FP64 vectors, products and scalars; x returned
    in FP32) against the oracle at every iteration.  FP64 rounding is
    amplified like FP32's but from 1e-16: the FP64 envelope (16 runs, each
    with its own perturbation of the sums, eps = u64 sqrt(L) / 3, and of the
    chord lengths, N(0,1) N u64 per entry: both tracers difference ray or
    offset parameters of magnitude up to about N, so their lengths carry
    absolute rounding of that order) grows about tenfold per iteration.  Up
    to the fixed count the iterate stays within the FP32 rounding of the
    returned x (2 u32) plus twice that envelope, where FP32 CGLS deviates by
    percents.  Near the end the oracle's own rounding, amplified, is of the
    envelope's size, so a slice where it dominates deviates by the same
    amount in the GPU run and in every envelope run."""
    from cgls_envelope import envelope_history
    A = gpu_matrix(N, M, C, "f64")
    Ao, ATo, _, y = cgls_problem(N, M, C, B)
    yd = y.double().numpy().reshape(B, -1)
    xg, resg, stg = gpu_cgls_history(A, y.cuda(), iters)
    xo, reso, sto, xho = oracle.cgls(Ao, ATo, yd, iters, history=True)
    L = max(Ao.nnz / Ao.shape[0], ATo.nnz / ATo.shape[0])
    env_x, env_r = envelope_history(Ao, ATo, yd, xho, reso, iters, storage="f64", seeds=range(16),
                                    eps=2.0 ** -53 * math.sqrt(L) / 3.0, entry_sd=2.0 ** -53 * N)
    u32 = 2.0 ** -24
    for k in range(1, iters + 1):
        dx = rel_err(xg[k - 1], xho[k - 1])
        dr = np.abs(resg[k] - reso[k]) / reso[k]
        banner(f"  f64 cgls N={N} k={k:2d} x dev {dx.max():.2e} (envelope {env_x[k].max():.2e}) "
               f"resid dev {dr.max():.2e}")
        assert np.all(dx <= 2 * u32 + 2 * env_x[k]), (k, dx)
        assert np.all(dr <= 1e-10 + 2 * env_r[k]), (k, dr)
    assert np.all(stg == sto)


@pytest.mark.parametrize("dt,opts,B", [("f32", {}, 5), ("f16", {}, 5), ("bf16", {}, 5), ("f64", {}, 5),
                                        ("f32", dict(tile_waves=32), 5), ("f16", dict(tile_waves=32), 5),
                                        ("f16", dict(fuse=32), 33), ("f32", dict(fuse=4, lds_bytes=32768), 5),
                                        ("f32", dict(fuse=1), 2), ("f16", dict(fuse=2), 3),
                                        ("f32", dict(stage_order=1), 5), ("f64", dict(fuse=2), 3)])
def test_lds_poison_build_is_bitwise_equal(dt, opts, B):
    """The debug build option that fills every stage buffer with NaN before
    the stage is copied in: if any entry read a slot its stage did not stage
    (a wrong slot, a tile copied late or into the wrong place, a stage
    barrier missing), its row would turn NaN.  Both products must equal the
    plain build's bit for bit."""
    N, M, C = 64, 90, 64
    banner(f"lds poison {dt} {opts} B={B}")
    A0 = gpu_matrix(N, M, C, dt, **opts)
    A1 = gpu_matrix(N, M, C, dt, debug_poison_lds=1, **opts)
    tdt = torch.float64 if dt == "f64" else torch.float32
    x = phantoms.ellipse_batch(N, B, 6, seed=77).to(tdt).cuda()
    y0, y1 = xct.project(A0, x), xct.project(A1, x)
    assert bool(torch.isfinite(y1).all())
    assert torch.equal(y0, y1)
    b0, b1 = xct.backproject(A0, y0), xct.backproject(A1, y0)
    assert bool(torch.isfinite(b1).all())
    assert torch.equal(b0, b1)
