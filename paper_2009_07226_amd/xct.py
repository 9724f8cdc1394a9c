"""Python binding of the C ABI in include/xct.h (ctypes; argument marshalling only).

Every step of projection, backprojection and CGLS runs in the HIP kernels of
libxct.so; torch supplies device memory and the current stream.  If the
library is missing, every call raises instead of computing anything on the
host.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxct.so")

F32, F16, BF16, F64 = 0, 1, 2, 3
_TORCH_DT = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16, torch.float64: F64}
_NAME_DT = {"f32": F32, "float32": F32, "f16": F16, "float16": F16, "bf16": BF16, "bfloat16": BF16,
            "f64": F64, "float64": F64}

EXPORTS = ("xct_build_matrix", "xct_free_matrix", "xct_matrix_info", "xct_spmm_workspace_bytes",
           "xct_project", "xct_backproject", "xct_cgls_workspace_bytes", "xct_cgls",
           "xct_matrix_to_coo", "xct_profile_enable", "xct_profile_read", "xct_last_error")


class XctError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"xct error {code}: {msg}")
        self.code = code


class BuildOpts(ctypes.Structure):
    _fields_ = [("tile_waves", ctypes.c_int), ("fuse", ctypes.c_int), ("lds_bytes", ctypes.c_int),
                ("xcd_remap", ctypes.c_int), ("stage_order", ctypes.c_int),
                ("lane_order", ctypes.c_int), ("slab_order", ctypes.c_int), ("arith", ctypes.c_int),
                ("debug_poison_lds", ctypes.c_int)]


class OpStats(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("padded", ctypes.c_int64), ("bytes", ctypes.c_int64),
                ("stages", ctypes.c_int64), ("staged_slots", ctypes.c_int64), ("blocks", ctypes.c_int32),
                ("tiles_per_stage", ctypes.c_int32), ("slabs", ctypes.c_int64), ("balanced_slabs", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MatrixInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("n_angles", ctypes.c_int), ("n_channels", ctypes.c_int),
                ("value_dtype", ctypes.c_int), ("fuse", ctypes.c_int), ("A", OpStats), ("AT", OpStats),
                ("build_seconds", ctypes.c_double)]


_lib = None


def library_loaded() -> bool:
    return _lib is not None


def lib():
    """Load libxct.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    L.xct_build_matrix.argtypes = [i, i, i, i, ctypes.POINTER(BuildOpts), vp, ctypes.POINTER(vp)]
    L.xct_build_matrix.restype = i
    L.xct_free_matrix.argtypes = [vp]
    L.xct_free_matrix.restype = None
    L.xct_matrix_info.argtypes = [vp, ctypes.POINTER(MatrixInfo)]
    L.xct_matrix_info.restype = i
    L.xct_spmm_workspace_bytes.argtypes = [vp, i]
    L.xct_spmm_workspace_bytes.restype = sz
    L.xct_project.argtypes = [vp, vp, vp, i, i, vp, vp]
    L.xct_project.restype = i
    L.xct_backproject.argtypes = [vp, vp, vp, i, i, vp, vp]
    L.xct_backproject.restype = i
    L.xct_cgls_workspace_bytes.argtypes = [vp, i, i]
    L.xct_cgls_workspace_bytes.restype = sz
    L.xct_cgls.argtypes = [vp, vp, i, vp, i, i, vp, vp, vp, vp]
    L.xct_cgls.restype = i
    L.xct_matrix_to_coo.argtypes = [vp, i, vp, vp, vp, i64, ctypes.POINTER(i64)]
    L.xct_matrix_to_coo.restype = i
    L.xct_profile_enable.argtypes = [i]
    L.xct_profile_enable.restype = i
    L.xct_profile_read.argtypes = [vp, vp]
    L.xct_profile_read.restype = i
    L.xct_read_bandwidth.argtypes = [vp, i64, i, ctypes.POINTER(ctypes.c_double), vp]
    L.xct_read_bandwidth.restype = i
    L.xct_stream_workspace_bytes.argtypes = [vp, i, i, i]
    L.xct_stream_workspace_bytes.restype = sz
    L.xct_project_streamed.argtypes = [vp, vp, vp, i, i, i, vp, vp, vp, vp]
    L.xct_project_streamed.restype = i
    L.xct_backproject_streamed.argtypes = [vp, vp, vp, i, i, i, vp, vp, vp, vp]
    L.xct_backproject_streamed.restype = i
    L.xct_pgrad_workspace_bytes.argtypes = [vp, i]
    L.xct_pgrad_workspace_bytes.restype = sz
    L.xct_projected_gradient.argtypes = [vp, vp, vp, i, i, vp, ctypes.c_float, ctypes.c_float, i, vp, vp]
    L.xct_projected_gradient.restype = i
    L.xct_count_nonfinite.argtypes = [vp, i64, i, vp, vp]
    L.xct_count_nonfinite.restype = i
    L.xct_device_memory.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.xct_device_memory.restype = i
    L.xct_last_error.argtypes = []
    L.xct_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(code: int):
    if code != 0:
        raise XctError(code, lib().xct_last_error().decode())


def _stream(stream=None) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dt(d) -> int:
    if isinstance(d, int):
        return d
    if isinstance(d, torch.dtype):
        return _TORCH_DT[d]
    return _NAME_DT[d]


def _require(t: torch.Tensor, shape, name: str, dtype=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU device")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dtype not in _TORCH_DT:
        raise TypeError(f"{name}: unsupported dtype {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _require_workspace(ws: torch.Tensor, nbytes: int, device: torch.device):
    """A caller-supplied workspace must be a contiguous device tensor of at
    least ``nbytes`` bytes on the matrix's device (the C ABI takes no size)."""
    if not isinstance(ws, torch.Tensor):
        raise TypeError("workspace must be a torch.Tensor")
    if ws.device != device:
        raise ValueError(f"workspace must be on {device}, got {ws.device}")
    if not ws.is_contiguous():
        raise ValueError("workspace must be contiguous")
    have = ws.numel() * ws.element_size()
    if have < nbytes:
        raise ValueError(f"workspace holds {have} bytes, the call needs {nbytes}")


class Matrix:
    """Handle of a built system matrix (A and A^T) resident on the current GPU."""

    def __init__(self, n: int, n_angles: int, n_channels: Optional[int] = None, dtype="f32", *,
                 tile_waves: int = 0, fuse: int = 0, lds_bytes: int = 0, xcd_remap: int = 0, stage_order: int = 0,
                 lane_order: int = 0, slab_order: int = 0, arith: int = 0, debug_poison_lds: int = 0,
                 stream=None):
        L = lib()
        n_channels = n if n_channels is None else n_channels
        self.n, self.n_angles, self.n_channels = int(n), int(n_angles), int(n_channels)
        self.value_dtype = _dt(dtype)
        self.device = torch.device("cuda", torch.cuda.current_device())
        opts = BuildOpts(int(tile_waves), int(fuse), int(lds_bytes), int(xcd_remap), int(stage_order),
                         int(lane_order), int(slab_order), int(arith), int(debug_poison_lds))
        h = ctypes.c_void_p()
        _check(L.xct_build_matrix(self.n, self.n_angles, self.n_channels, self.value_dtype, ctypes.byref(opts),
                                  _stream(stream), ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("matrix has been freed")
        return self._h

    def free(self):
        if getattr(self, "_h", None) is not None:
            torch.cuda.synchronize(self.device)
            lib().xct_free_matrix(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self) -> dict:
        mi = MatrixInfo()
        _check(lib().xct_matrix_info(self.handle, ctypes.byref(mi)))
        return {"n": mi.n, "n_angles": mi.n_angles, "n_channels": mi.n_channels, "value_dtype": mi.value_dtype,
                "fuse": mi.fuse, "A": mi.A.as_dict(), "AT": mi.AT.as_dict(), "build_seconds": mi.build_seconds}

    def to_coo(self, which: int = 0):
        """Decode A (which=0) or A^T (which=1) to host COO arrays (rows, cols, vals)."""
        info = self.info()
        cap = info["AT" if which else "A"]["nnz"]
        rows = np.empty(max(cap, 1), np.int32)
        cols = np.empty(max(cap, 1), np.int32)
        vals = np.empty(max(cap, 1), np.float32)
        cnt = ctypes.c_int64()
        _check(lib().xct_matrix_to_coo(self.handle, int(which), rows.ctypes.data, cols.ctypes.data,
                                       vals.ctypes.data, cap, ctypes.byref(cnt)))
        k = cnt.value
        return rows[:k], cols[:k], vals[:k]

    @property
    def vol_shape(self):
        return (self.n, self.n)

    @property
    def sino_shape(self):
        return (self.n_angles, self.n_channels)

    def spmm_workspace(self, batch: int) -> torch.Tensor:
        nb = lib().xct_spmm_workspace_bytes(self.handle, int(batch))
        return torch.empty(nb, dtype=torch.uint8, device=self.device)

    def cgls_workspace(self, batch: int, iters: int) -> torch.Tensor:
        nb = lib().xct_cgls_workspace_bytes(self.handle, int(batch), int(iters))
        return torch.empty(nb, dtype=torch.uint8, device=self.device)


def project(A: Matrix, x: torch.Tensor, out: Optional[torch.Tensor] = None,
            workspace: Optional[torch.Tensor] = None, check_finite: bool = False) -> torch.Tensor:
    """y = A x for a batch x of shape (B, n, n); returns (B, n_angles, n_channels) in x's dtype.
    With ``check_finite``, raise ValueError if x holds a NaN or an infinity."""
    B = x.shape[0] if x.dim() == 3 else -1
    _require(x, (B,) + A.vol_shape, "x")
    if check_finite and count_nonfinite(x):
        raise ValueError("x holds non-finite values")
    if out is None:
        out = torch.empty((B,) + A.sino_shape, dtype=x.dtype, device=x.device)
    _require(out, (B,) + A.sino_shape, "out", x.dtype)
    if workspace is None:
        workspace = A.spmm_workspace(B)
    else:
        _require_workspace(workspace, lib().xct_spmm_workspace_bytes(A.handle, B), A.device)
    _check(lib().xct_project(A.handle, x.data_ptr(), out.data_ptr(), B, _dt(x.dtype), workspace.data_ptr(),
                             _stream()))
    return out


def backproject(A: Matrix, y: torch.Tensor, out: Optional[torch.Tensor] = None,
                workspace: Optional[torch.Tensor] = None, check_finite: bool = False) -> torch.Tensor:
    """x = A^T y for a batch y of shape (B, n_angles, n_channels); returns (B, n, n).
    With ``check_finite``, raise ValueError if y holds a NaN or an infinity."""
    B = y.shape[0] if y.dim() == 3 else -1
    _require(y, (B,) + A.sino_shape, "y")
    if check_finite and count_nonfinite(y):
        raise ValueError("y holds non-finite values")
    if out is None:
        out = torch.empty((B,) + A.vol_shape, dtype=y.dtype, device=y.device)
    _require(out, (B,) + A.vol_shape, "out", y.dtype)
    if workspace is None:
        workspace = A.spmm_workspace(B)
    else:
        _require_workspace(workspace, lib().xct_spmm_workspace_bytes(A.handle, B), A.device)
    _check(lib().xct_backproject(A.handle, y.data_ptr(), out.data_ptr(), B, _dt(y.dtype), workspace.data_ptr(),
                                 _stream()))
    return out


def _require_host(t: torch.Tensor, shape, name: str, dtype=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cpu":
        raise ValueError(f"{name} must be in host memory")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dtype not in _TORCH_DT:
        raise TypeError(f"{name}: unsupported dtype {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


_COPY_STREAMS = {}


def _copy_streams(device):
    # two copy streams per device (host-to-device, device-to-host), default priority
    if device not in _COPY_STREAMS:
        _COPY_STREAMS[device] = (torch.cuda.Stream(device=device), torch.cuda.Stream(device=device))
    return _COPY_STREAMS[device]


def _streamed(which: int, A: Matrix, src: torch.Tensor, out: Optional[torch.Tensor], chunk: Optional[int],
              workspace: Optional[torch.Tensor]) -> torch.Tensor:
    in_shape, out_shape = (A.vol_shape, A.sino_shape) if which == 0 else (A.sino_shape, A.vol_shape)
    B = src.shape[0] if src.dim() == 3 else -1
    _require_host(src, (B,) + in_shape, "input")
    if out is None:
        out = torch.empty((B,) + out_shape, dtype=src.dtype, pin_memory=True)
    _require_host(out, (B,) + out_shape, "out", src.dtype)
    chunk = int(chunk) if chunk else 16
    nb = lib().xct_stream_workspace_bytes(A.handle, which, chunk, _dt(src.dtype))
    if workspace is None:
        workspace = torch.empty(nb, dtype=torch.uint8, device=A.device)
    else:
        _require_workspace(workspace, nb, A.device)
    h2d, d2h = _copy_streams(A.device)
    fn = lib().xct_project_streamed if which == 0 else lib().xct_backproject_streamed
    _check(fn(A.handle, src.data_ptr(), out.data_ptr(), B, chunk, _dt(src.dtype), workspace.data_ptr(),
              _stream(), _stream(h2d), _stream(d2h)))
    return out


def project_streamed(A: Matrix, x: torch.Tensor, out: Optional[torch.Tensor] = None, chunk: Optional[int] = None,
                     workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = A x for a host batch x of shape (B, n, n) (page-locked for overlap), moved to
    the GPU `chunk` slices at a time; returns a host (B, n_angles, n_channels) tensor."""
    return _streamed(0, A, x, out, chunk, workspace)


def backproject_streamed(A: Matrix, y: torch.Tensor, out: Optional[torch.Tensor] = None,
                         chunk: Optional[int] = None, workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = A^T y for a host batch y of shape (B, n_angles, n_channels), streamed as
    project_streamed; returns a host (B, n, n) tensor."""
    return _streamed(1, A, y, out, chunk, workspace)


def cgls(A: Matrix, y: torch.Tensor, iters: int, out: Optional[torch.Tensor] = None,
         workspace: Optional[torch.Tensor] = None, want_resid: bool = True):
    """Per-slice CGLS from zero for `iters` iterations.  Returns (x (B, n, n) FP32,
    resid (iters+1, B) numpy or None, status (B,) numpy or None)."""
    B = y.shape[0] if y.dim() == 3 else -1
    _require(y, (B,) + A.sino_shape, "y")
    if out is None:
        out = torch.empty((B,) + A.vol_shape, dtype=torch.float32, device=y.device)
    _require(out, (B,) + A.vol_shape, "out", torch.float32)
    if workspace is None:
        workspace = A.cgls_workspace(B, iters)
    else:
        _require_workspace(workspace, lib().xct_cgls_workspace_bytes(A.handle, B, int(iters)), A.device)
    resid = np.empty((iters + 1, B), np.float64) if want_resid else None
    status = np.empty(B, np.int32) if want_resid else None
    _check(lib().xct_cgls(A.handle, y.data_ptr(), _dt(y.dtype), out.data_ptr(), B, int(iters),
                          workspace.data_ptr(), resid.ctypes.data if want_resid else None,
                          status.ctypes.data if want_resid else None, _stream()))
    return out, resid, status


def projected_gradient(A: Matrix, y: torch.Tensor, iters: int, step, lam: float = 0.0, eps: float = 1e-2,
                       nonneg: bool = True, x0: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                       workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Projected gradient descent on ||y - A x||^2 + lam * TV_eps(x) over x >= 0
    (or all x when ``nonneg`` is False), `iters` iterations from x0 (zero when
    None).  y: (B, n_angles, n_channels) FP32; step: a float or a (B,) tensor of
    per-slice steps.  Returns x (B, n, n) FP32 (``out`` when given)."""
    B = y.shape[0] if y.dim() == 3 else -1
    _require(y, (B,) + A.sino_shape, "y", torch.float32)
    if iters < 0 or not eps > 0.0 or not lam >= 0.0:
        raise ValueError("need iters >= 0, eps > 0 and lam >= 0")
    if out is None:
        out = torch.empty((B,) + A.vol_shape, dtype=torch.float32, device=y.device)
    _require(out, (B,) + A.vol_shape, "out", torch.float32)
    if x0 is None:
        out.zero_()
    else:
        _require(x0, (B,) + A.vol_shape, "x0", torch.float32)
        if x0.data_ptr() != out.data_ptr():
            out.copy_(x0)
    if isinstance(step, torch.Tensor):
        tau = step.to(device=y.device, dtype=torch.float32).reshape(-1).contiguous()
        if tau.numel() != B:
            raise ValueError(f"step has {tau.numel()} entries, expected {B}")
    else:
        tau = torch.full((B,), float(step), dtype=torch.float32, device=y.device)
    nb = lib().xct_pgrad_workspace_bytes(A.handle, B)
    if workspace is None:
        workspace = torch.empty(nb, dtype=torch.uint8, device=y.device)
    else:
        _require_workspace(workspace, nb, A.device)
    _check(lib().xct_projected_gradient(A.handle, y.data_ptr(), out.data_ptr(), B, int(iters), tau.data_ptr(),
                                        float(lam), float(eps), 1 if nonneg else 0, workspace.data_ptr(), _stream()))
    return out


def count_nonfinite(t: torch.Tensor) -> int:
    """Number of NaN / infinite elements of a contiguous device tensor
    (FP32, FP16 or BF16); waits for the count."""
    _require(t, tuple(t.shape), "tensor")
    c = torch.empty((), dtype=torch.int64, device=t.device)
    _check(lib().xct_count_nonfinite(t.data_ptr(), t.numel(), _dt(t.dtype), c.data_ptr(), _stream()))
    return int(c.item())


def device_memory() -> dict:
    """Device buffers (count and bytes) the library holds for its matrices."""
    n, b = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().xct_device_memory(ctypes.byref(n), ctypes.byref(b)))
    return {"buffers": n.value, "bytes": b.value}


def profile_enable(on: bool = True) -> None:
    """Bracket every SpMM kernel launch with HIP events (measurement only)."""
    _check(lib().xct_profile_enable(1 if on else 0))


def profile_read() -> dict:
    """Launch counts and total kernel milliseconds per operator since the last read."""
    n = np.zeros(2, np.int64)
    ms = np.zeros(2, np.float64)
    _check(lib().xct_profile_read(n.ctypes.data, ms.ctypes.data))
    return {"A": (int(n[0]), float(ms[0])), "AT": (int(n[1]), float(ms[1]))}


def read_bandwidth(buf: torch.Tensor, reps: int = 5, stream=None) -> float:
    """Streaming-read GB/s of the device over a resident tensor (measurement utility)."""
    if not buf.is_cuda or not buf.is_contiguous():
        raise ValueError("buf must be a contiguous CUDA tensor")
    g = ctypes.c_double()
    _check(lib().xct_read_bandwidth(buf.data_ptr(), buf.numel() * buf.element_size(), int(reps), ctypes.byref(g),
                                    _stream(stream)))
    return g.value


class XctProject(torch.autograd.Function):
    """y = A x with backward g -> A^T g (the hand-written backprojection)."""

    @staticmethod
    def forward(ctx, x, A):
        ctx.A = A
        return project(A, x.contiguous())

    @staticmethod
    def backward(ctx, g):
        return XctBackproject.apply(g.contiguous(), ctx.A), None


class XctBackproject(torch.autograd.Function):
    """x = A^T y with backward g -> A g (the hand-written projection)."""

    @staticmethod
    def forward(ctx, y, A):
        ctx.A = A
        return backproject(A, y.contiguous())

    @staticmethod
    def backward(ctx, g):
        return XctProject.apply(g.contiguous(), ctx.A), None
