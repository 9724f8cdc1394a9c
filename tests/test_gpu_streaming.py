"""Slice streaming on one GPU (host-resident batches moved in chunks on copy
streams, overlapped with the SpMM): results equal the device-resident entry
points on the same slices, and match the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2009_07226_amd import phantoms
from paper_2009_07226_amd import xct

pytestmark = pytest.mark.gpu


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def rel_err(a, b):
    a = np.asarray(a, np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, np.float64).reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


@pytest.mark.parametrize("dt", ["f32", "f16"])
@pytest.mark.parametrize("B,chunk", [(37, 16), (37, 10), (5, 16), (1, 1), (20, 3)])
def test_streamed_equals_device_calls(dt, B, chunk):
    banner(f"streamed {dt} B={B} chunk={chunk}")
    N, M, C = 64, 90, 64
    A = xct.Matrix(N, M, C, dt)
    x = phantoms.ellipse_batch(N, B, 6, seed=7 + B).float().pin_memory()
    y_dev = xct.project(A, x.cuda())
    y_str = xct.project_streamed(A, x, chunk=chunk)
    assert y_str.device.type == "cpu"
    # per-slice sums and per-slice operand scaling do not depend on the chunking
    assert torch.equal(y_str, y_dev.cpu())
    yp = y_dev.cpu().pin_memory()
    xb_dev = xct.backproject(A, y_dev)
    xb_str = xct.backproject_streamed(A, yp, chunk=chunk)
    assert torch.equal(xb_str, xb_dev.cpu())


def test_streamed_waits_for_earlier_work_on_the_compute_stream():
    # The workspace of a streamed call may be memory the caching allocator just
    # took back from a product still running on the compute stream; the copy
    # streams must not write it before that product is done.
    N, M, C, B = 128, 180, 128, 16
    A = xct.Matrix(N, M, C, "f32")
    x = phantoms.ellipse_batch(N, B, 6, seed=11).float()
    xd = x.cuda()
    ref = xct.project(A, xd).cpu()
    xh = x.pin_memory()
    for _ in range(3):
        y_dev = xct.project(A, xd)  # its workspace is released while the kernels run
        y_str = xct.project_streamed(A, xh, chunk=4)
        assert torch.equal(y_dev.cpu(), ref)
        assert torch.equal(y_str, ref)


def test_streamed_matches_oracle_fp16_io():
    N, M, C, B = 48, 40, 50, 9
    A = xct.Matrix(N, M, C, "f32")
    Ao = oracle.build_A(N, M, C)
    x = phantoms.ellipse_batch(N, B, 5, seed=3).float()
    y = xct.project_streamed(A, x.pin_memory(), chunk=4)
    assert rel_err(y.numpy(), oracle.project(Ao, x.double().numpy().reshape(B, -1))).max() <= 1e-5
    # 16-bit host io: the storage rounding of the operand and the result
    y16 = xct.project_streamed(A, x.half().pin_memory(), chunk=4)
    assert y16.dtype == torch.float16
    assert rel_err(y16.float().numpy(), oracle.project(Ao, x.double().numpy().reshape(B, -1))).max() <= 2e-3


def test_streamed_argument_checks():
    A = xct.Matrix(16, 12, 16, "f32")
    with pytest.raises(ValueError):
        xct.project_streamed(A, torch.zeros(2, 16, 16, device="cuda"))
    with pytest.raises(ValueError):
        xct.project_streamed(A, torch.zeros(2, 15, 16))
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    L = xct.lib()
    x = torch.zeros(2, 16, 16).pin_memory()
    y = torch.zeros(2, 12, 16).pin_memory()
    # chunk < 1
    assert L.xct_project_streamed(A.handle, x.data_ptr(), y.data_ptr(), 2, 0, 0, ws.data_ptr(), None, None,
                                  None) == -1
    assert b"chunk" in L.xct_last_error()
    # misaligned workspace
    assert L.xct_project_streamed(A.handle, x.data_ptr(), y.data_ptr(), 2, 1, 0, ws.data_ptr() + 4, None, None,
                                  None) == -1
