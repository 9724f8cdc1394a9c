"""The allocation-free form of the products (xct_apply_noalloc): the same
results as xct_project / xct_backproject with a caller workspace, bit for bit
(every slice's sums are the same for any number of fused slices), on two
calls in a row whose second input is smaller, and a clear error where one
slice's staging exceeds the fixed scratch array."""
import ctypes

import pytest
import torch

pytestmark = pytest.mark.gpu

xct = pytest.importorskip("paper_2009_07226_amd")


def noalloc(A, which, src, out):
    L = xct.lib()
    L.xct_apply_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_void_p]
    L.xct_apply_noalloc.restype = ctypes.c_int
    io = {torch.float32: 0, torch.float16: 1, torch.bfloat16: 2, torch.float64: 3}[src.dtype]
    rc = L.xct_apply_noalloc(A.handle, which, src.data_ptr(), out.data_ptr(), src.shape[0], io,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise xct.XctError(rc, L.xct_last_error().decode())
    return out


@pytest.mark.parametrize("dt,io,kw,batches", [("f32", torch.float32, {}, (17, 3)),
                                              ("f16", torch.float16, {}, (17, 3)),
                                              ("bf16", torch.float32, {}, (17, 3)),
                                              ("f64", torch.float64, {}, (17, 3)),
                                              ("f16", torch.float32, {"fuse": 32}, (40, 5))])
def test_noalloc_equals_workspace_products(dt, io, kw, batches):
    from paper_2009_07226_amd import phantoms
    A = xct.Matrix(128, 180, 128, dt, **kw)
    for B in batches:  # the second call's input is smaller
        x = phantoms.ellipse_batch(128, B, 6, seed=B).to("cuda", io)
        y_ref = xct.project(A, x)
        y = noalloc(A, 0, x, torch.full_like(y_ref, float("nan")))
        assert torch.equal(y, y_ref)
        xb_ref = xct.backproject(A, y_ref)
        xb = noalloc(A, 1, y_ref, torch.full_like(xb_ref, float("nan")))
        assert torch.equal(xb, xb_ref)
    torch.cuda.synchronize()
    A.free()


def test_noalloc_smaller_matrix_after_larger():
    from paper_2009_07226_amd import phantoms
    for n, m in ((300, 200), (37, 23)):
        A = xct.Matrix(n, m, n, "f32")
        x = phantoms.ellipse_batch(n, 5, 4, seed=n).cuda().float()
        y = noalloc(A, 0, x, torch.empty((5, m, n), device="cuda"))
        assert torch.equal(y, xct.project(A, x))
        xb = noalloc(A, 1, y, torch.empty((5, n, n), device="cuda"))
        assert torch.equal(xb, xct.backproject(A, y))
        torch.cuda.synchronize()
        A.free()


def test_noalloc_rejects_geometry_beyond_scratch():
    L = xct.lib()
    L.xct_noalloc_scratch_bytes.restype = ctypes.c_size_t
    cap = L.xct_noalloc_scratch_bytes()
    n = 4096  # one FP32 slice stages 4096^2 / 64 tiles x 64 x 8 bytes = 128 MiB
    assert (n * n * 8) > cap
    A = xct.Matrix(n, 4, n, "f32")
    x = torch.zeros((1, n, n), device="cuda")
    with pytest.raises(xct.XctError) as e:
        noalloc(A, 0, x, torch.empty((1, 4, n), device="cuda"))
    assert e.value.code == -4 and "scratch" in str(e.value)
    A.free()
