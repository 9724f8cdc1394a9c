"""FP64 CPU oracle for parallel-beam XCT (projection, backprojection, CGLS).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product
library (``paper_2009_07226_amd``) never imports it and shares no code with
it.

What it computes follows Hidayetoglu et al., "Petascale XCT" (SC20):
Eq. (1) with R = 0 (least squares), the parallel-beam Siddon system matrix
of Sec. II-A shared by every slice (Sec. II-B), and CGLS from x0 = 0 with a
fixed iteration count (Sec. IV-F; Table IV note: k iterations are k
projections and k+1 backprojections).  The geometry readings (grid, angles,
detector offsets, edge rule) are stated in ``xct_oracle.c``.

Pins (see tests/test_oracle_pins.py): analytic chord lengths of the whole
grid, axis-aligned rays, voxel-aligned rectangles, disc projections under
refinement, a hand-derived 2x2 example, brute force over all ray/voxel
pairs, the adjoint identity between the ray-driven and the voxel-driven
builds, rotation/reflection symmetries, and CGLS against Krylov least
squares by dense QR and against the minimum-norm lstsq solution; the
per-iteration history (``cgls(..., history=True)``) and the A-only form for
scans too large for both matrices (``TracedA``: A^T as A's transposed
product) against the same Krylov solutions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "xct_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_intp = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")


def build_library(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
             "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build_library(force=True)
    lib = ctypes.CDLL(_LIB)
    I, L = ctypes.c_int, ctypes.c_int64
    lib.oracle_siddon_row.argtypes = [I, I, I, L, _i32p, _f64p]
    lib.oracle_siddon_row.restype = L
    lib.oracle_voxel_col.argtypes = [I, I, I, L, _i32p, _f64p]
    lib.oracle_voxel_col.restype = L
    lib.oracle_counts_A.argtypes = [I, I, I, _i64p]
    lib.oracle_fill_A.argtypes = [I, I, I, _i64p, _i32p, _f64p]
    lib.oracle_counts_AT.argtypes = [I, I, I, _i64p]
    lib.oracle_fill_AT.argtypes = [I, I, I, _i64p, _i32p, _f64p]
    lib.oracle_csr_spmm.argtypes = [L, _i64p, _i32p, _f64p, L, I, _f64p, _f64p]
    lib.oracle_project_rows.argtypes = [I, I, I, I, _f64p, L, _i64p, _f64p]
    lib.oracle_backproject_voxels.argtypes = [I, I, I, I, _f64p, L, _i64p, _f64p]
    _f64p_or_null = ctypes.c_void_p
    lib.oracle_cgls.argtypes = [L, _i64p, _i32p, _f64p, L, _i64p, _i32p, _f64p,
                                I, _f64p, I, _f64p, _f64p, _intp, _f64p_or_null]
    lib.oracle_traced_build.argtypes = [I, I, I]
    lib.oracle_traced_build.restype = ctypes.c_void_p
    lib.oracle_traced_nnz.argtypes = [ctypes.c_void_p]
    lib.oracle_traced_nnz.restype = L
    lib.oracle_traced_project.argtypes = [ctypes.c_void_p, I, _f64p, _f64p]
    lib.oracle_traced_project.restype = None
    lib.oracle_traced_backproject.argtypes = [ctypes.c_void_p, I, _f64p, _f64p]
    lib.oracle_traced_backproject.restype = None
    lib.oracle_traced_cgls.argtypes = [ctypes.c_void_p, I, _f64p, I, _f64p, _f64p, _intp, _f64p_or_null]
    lib.oracle_traced_cgls.restype = None
    lib.oracle_traced_free.argtypes = [ctypes.c_void_p]
    lib.oracle_traced_free.restype = None
    for f in ("oracle_counts_A", "oracle_fill_A", "oracle_counts_AT", "oracle_fill_AT",
              "oracle_csr_spmm", "oracle_project_rows", "oracle_backproject_voxels", "oracle_cgls"):
        getattr(lib, f).restype = None
    _lib = lib
    return lib


def set_threads(n: int) -> None:
    """Thread count for the OpenMP loops (applies to the next parallel region)."""
    os.environ["OMP_NUM_THREADS"] = str(int(n))
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    except OSError:
        pass


# ---- entries ----------------------------------------------------------------

def siddon_row(N: int, M: int, C: int, r: int):
    """Row r = k*C + c of A, ray-driven (Siddon).  Returns (cols, vals)."""
    lib = _load()
    cols = np.empty(2 * N + 2, np.int32)
    vals = np.empty(2 * N + 2, np.float64)
    n = lib.oracle_siddon_row(N, M, C, r, cols, vals)
    return cols[:n].copy(), vals[:n].copy()


def voxel_col(N: int, M: int, C: int, v: int):
    """Column v = i*N + j of A, voxel-driven.  Returns (rows, vals)."""
    lib = _load()
    rows = np.empty(4 * M, np.int32)
    vals = np.empty(4 * M, np.float64)
    n = lib.oracle_voxel_col(N, M, C, v, rows, vals)
    return rows[:n].copy(), vals[:n].copy()


def build_A(N: int, M: int, C: int) -> sp.csr_matrix:
    """A as an (M*C) x (N*N) CSR matrix, traced ray by ray (Siddon)."""
    lib = _load()
    R = M * C
    counts = np.empty(R, np.int64)
    lib.oracle_counts_A(N, M, C, counts)
    ptr = np.zeros(R + 1, np.int64)
    np.cumsum(counts, out=ptr[1:])
    cols = np.empty(int(ptr[-1]), np.int32)
    vals = np.empty(int(ptr[-1]), np.float64)
    lib.oracle_fill_A(N, M, C, ptr, cols, vals)
    return sp.csr_matrix((vals, cols, ptr), shape=(R, N * N))


def build_AT(N: int, M: int, C: int) -> sp.csr_matrix:
    """A^T as an (N*N) x (M*C) CSR matrix, built voxel by voxel."""
    lib = _load()
    V = N * N
    counts = np.empty(V, np.int64)
    lib.oracle_counts_AT(N, M, C, counts)
    ptr = np.zeros(V + 1, np.int64)
    np.cumsum(counts, out=ptr[1:])
    rows = np.empty(int(ptr[-1]), np.int32)
    vals = np.empty(int(ptr[-1]), np.float64)
    lib.oracle_fill_AT(N, M, C, ptr, rows, vals)
    return sp.csr_matrix((vals, rows, ptr), shape=(V, M * C))


def _csr_parts(m: sp.csr_matrix):
    return (np.ascontiguousarray(m.indptr, dtype=np.int64),
            np.ascontiguousarray(m.indices, dtype=np.int32),
            np.ascontiguousarray(m.data, dtype=np.float64))


# ---- products -----------------------------------------------------------------

def spmm(m: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """Y[b] = m @ X[b] for a batch X of shape (B, ncols), in FP64."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    squeeze = x.ndim == 1
    x2 = x.reshape(1 if squeeze else x.shape[0], -1)
    assert x2.shape[1] == m.shape[1]
    y = np.empty((x2.shape[0], m.shape[0]), np.float64)
    p, c, v = _csr_parts(m)
    lib.oracle_csr_spmm(m.shape[0], p, c, v, m.shape[1], x2.shape[0], x2, y)
    return y[0] if squeeze else y


def project(A: sp.csr_matrix, x: np.ndarray) -> np.ndarray:
    """Forward projection of a batch of slices x (B, N, N) -> (B, M*C)."""
    return spmm(A, np.asarray(x).reshape(np.asarray(x).shape[0], -1))


def backproject(AT: sp.csr_matrix, y: np.ndarray) -> np.ndarray:
    """Backprojection of a batch of sinograms y (B, M, C) -> (B, N*N)."""
    return spmm(AT, np.asarray(y).reshape(np.asarray(y).shape[0], -1))


def project_rows(N: int, M: int, C: int, x: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """(A x_b)[rows] for every slice b, tracing only the requested rays."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, N * N)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((x.shape[0], rows.size), np.float64)
    lib.oracle_project_rows(N, M, C, x.shape[0], x, rows.size, rows, out)
    return out


def backproject_voxels(N: int, M: int, C: int, y: np.ndarray, vox: np.ndarray) -> np.ndarray:
    """(A^T y_b)[vox] for every slice b, from voxel-driven columns."""
    lib = _load()
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(-1, M * C)
    vox = np.ascontiguousarray(vox, dtype=np.int64)
    out = np.empty((y.shape[0], vox.size), np.float64)
    lib.oracle_backproject_voxels(N, M, C, y.shape[0], y, vox.size, vox, out)
    return out


def cgls(A: sp.csr_matrix, AT: sp.csr_matrix, y: np.ndarray, iters: int, history: bool = False):
    """Per-slice CGLS from x0 = 0.  y: (B, M*C).  Returns (x (B, N*N),
    resid (iters+1, B) of ||r_k||/||y||, status (B,), 1 = stopped early), and
    with ``history`` also xhist (iters, B, N*N): x_k for k = 1..iters."""
    lib = _load()
    y = np.ascontiguousarray(y, dtype=np.float64).reshape(np.asarray(y).shape[0], -1)
    B = y.shape[0]
    x = np.empty((B, A.shape[1]), np.float64)
    resid = np.empty((iters + 1, B), np.float64)
    status = np.empty(B, np.int32)
    xh = np.empty((iters, B, A.shape[1]), np.float64) if history else None
    ap, ac, av = _csr_parts(A)
    tp, tc, tv = _csr_parts(AT)
    lib.oracle_cgls(A.shape[0], ap, ac, av, A.shape[1], tp, tc, tv, B, y, iters, x, resid, status,
                    xh.ctypes.data if history else None)
    return (x, resid, status, xh) if history else (x, resid, status)


class TracedA:
    """The scan (N, M, C) with only A held in host memory, as a CSR traced ray
    by ray inside the C library (12 bytes per entry); A^T is applied as A's
    transposed product.  For scans where A and A^T would not both fit.  Use as
    a context manager or call ``close``."""

    def __init__(self, N: int, M: int, C: int):
        self.N, self.M, self.C = N, M, C
        self._h = _load().oracle_traced_build(N, M, C)
        if not self._h:
            raise MemoryError("oracle_traced_build: the CSR of A does not fit in host memory")

    @property
    def nnz(self) -> int:
        return int(_load().oracle_traced_nnz(self._h))

    def project(self, x: np.ndarray) -> np.ndarray:
        """A x_b for x (B, N, N) or (B, N*N) -> (B, M*C)."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(np.asarray(x).shape[0], -1)
        assert x.shape[1] == self.N * self.N
        y = np.empty((x.shape[0], self.M * self.C), np.float64)
        _load().oracle_traced_project(self._h, x.shape[0], x, y)
        return y

    def backproject(self, w: np.ndarray) -> np.ndarray:
        """A^T w_b (the transposed product of A's rows) for w (B, M, C) or
        (B, M*C) -> (B, N*N)."""
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(np.asarray(w).shape[0], -1)
        assert w.shape[1] == self.M * self.C
        x = np.empty((w.shape[0], self.N * self.N), np.float64)
        _load().oracle_traced_backproject(self._h, w.shape[0], w, x)
        return x

    def cgls(self, y: np.ndarray, iters: int, history: bool = False):
        """Per-slice CGLS as ``cgls``; same returns."""
        y = np.ascontiguousarray(y, dtype=np.float64).reshape(np.asarray(y).shape[0], -1)
        B = y.shape[0]
        assert y.shape[1] == self.M * self.C
        nc = self.N * self.N
        x = np.empty((B, nc), np.float64)
        resid = np.empty((iters + 1, B), np.float64)
        status = np.empty(B, np.int32)
        xh = np.empty((iters, B, nc), np.float64) if history else None
        _load().oracle_traced_cgls(self._h, B, y, iters, x, resid, status, xh.ctypes.data if history else None)
        return (x, resid, status, xh) if history else (x, resid, status)

    def close(self):
        if self._h:
            _load().oracle_traced_free(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
