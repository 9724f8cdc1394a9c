"""Rounding envelope of CGLS iterates (test helper).

CGLS iterates are ill-conditioned under rounding: a perturbation of relative
size eps in every step grows through the recurrences, and after enough
iterations the iterate differs from the exact one by far more than eps.  This
helper measures that growth: it runs CGLS in the precision the GPU solver
stores and sums in, but with other summation orders, and returns per
iteration k the largest relative deviation of x_k and of the residual norm
from the FP64 oracle's exact history.  A GPU solver that rounds the same way
deviates by about as much; one that loses more precision deviates by more.

Each run ("order") works on the oracle's matrix (the FP64 chord lengths):
  * matrix values rounded to the storage format (FP32, FP16 or BF16),
    nearest even;
  * product operands: FP32 as stored; with 16-bit storage scaled per slice by
    the power of two m = 2^ceil(log2 max|v|) and rounded to 16 bits;
  * every row of every product summed in FP32 with one fused multiply-add
    per entry (fp32_spmm.c), the entries of each row taken cyclically from a
    hashed start, alternately forwards and backwards (a different order per
    run), stored in FP32;
  * solver vectors x, r, p stored in FP32 after every update, step lengths
    rounded to FP32 where they scale a vector, dot products in FP64.
``envelope_history(..., storage="f64")`` instead keeps everything in FP64
and adds eps * N(0,1) * (|A| |v|)_r to output r of every product A v (the
forward error of a dot product is proportional to the sum of its terms'
magnitudes; A is non-negative, so |A| |v| is the product of |v|): the
amplification study of the oracle pins, and the envelope of FP64 solvers.
With ``entry_sd`` every run also adds entry_sd * N(0,1) to each matrix
entry of A and of A^T (independently): the absolute rounding of chord
lengths that another FP64 tracer computes from the same geometry."""
import ctypes
import hashlib
import os
import subprocess
import tempfile

import numpy as np
import scipy.sparse as sp

import oracle

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


def _spmm_lib():
    """The FP32 product helper, compiled with gcc on first use."""
    global _lib
    if _lib is None:
        src = os.path.join(_HERE, "fp32_spmm.c")
        tag = hashlib.sha256(open(src, "rb").read()).hexdigest()[:12]
        so = os.path.join(tempfile.gettempdir(), f"xct_fp32_spmm_{tag}.so")
        if not os.path.exists(so):
            tmp = so + f".{os.getpid()}"
            subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", src,
                                   "-o", tmp, "-lm"])
            os.replace(tmp, so)
        lib = ctypes.CDLL(so)
        p = np.ctypeslib.ndpointer
        lib.fp32_csr_spmm.argtypes = [ctypes.c_int64, p(np.int64, flags="C"), p(np.int32, flags="C"),
                                      p(np.float32, flags="C"), ctypes.c_int64, ctypes.c_int,
                                      p(np.float32, flags="C"), p(np.float32, flags="C"), ctypes.c_int64]
        lib.fp32_csr_spmm.restype = None
        _lib = lib
    return _lib


def f32(v):
    return np.asarray(v, np.float64).astype(np.float32).astype(np.float64)


def bf16(v):
    """nearest-even rounding to BF16, through FP32 (exact for FP32-stored
    vectors; for the FP64 lengths a double rounding could differ from a
    direct one only in a tie of the FP32 value, which no length here hits)"""
    u = np.asarray(v, np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_to(v, storage):
    if storage == "f32":
        return f32(v)
    if storage == "f16":
        return np.asarray(v, np.float64).astype(np.float16).astype(np.float64)
    if storage == "bf16":
        return bf16(v)
    raise ValueError(storage)


class Fp32Product:
    """A CSR operator with values rounded to `storage`, applied in FP32
    (fp32_spmm.c) to a batch, summing each row in the order `order` picks."""

    def __init__(self, m: sp.csr_matrix, storage: str, order: int):
        m = m.tocsr()
        self.ptr = np.ascontiguousarray(m.indptr, np.int64)
        self.idx = np.ascontiguousarray(m.indices, np.int32)
        self.val = np.ascontiguousarray(round_to(m.data, storage), np.float32)
        self.shape, self.order = m.shape, int(order)

    def __call__(self, v):
        v32 = np.ascontiguousarray(v, np.float32)
        out = np.empty((v32.shape[0], self.shape[0]), np.float32)
        _spmm_lib().fp32_csr_spmm(self.shape[0], self.ptr, self.idx, self.val, self.shape[1], v32.shape[0], v32,
                                  out, self.order)
        return out.astype(np.float64)


def _pow2_ceil(mx):
    m = np.ones_like(mx)
    ok = (mx > 0) & np.isfinite(mx)
    m[ok] = 2.0 ** np.ceil(np.log2(mx[ok]))
    return m


def envelope_history(A, AT, y, xh_ref, res_ref, iters, storage="f32", seeds=(0, 1, 2), eps=0.0, entry_sd=0.0):
    """A, AT: the oracle's CSR pair.  y (B, rows); xh_ref (iters, B, cols):
    the oracle's x_1..x_iters; res_ref (iters+1, B): its residual history.
    storage: "f32", "f16" or "bf16" (the solver's arithmetic above), or
    "f64" (FP64 throughout, every product output perturbed by eps * N(0,1)
    * (|A| |v|)_r, the entries by entry_sd * N(0,1)).  Returns (env_x, env_r), each (iters+1, B): max over the
    seeded runs of ||x_k - x_k*|| / ||x_k*|| and of | r_k - r_k* | / r_k*
    (0 at k = 0, where both start from x = 0)."""
    y = np.asarray(y, np.float64)
    B = y.shape[0]
    env_x = np.zeros((iters + 1, B))
    env_r = np.zeros((iters + 1, B))
    for seed in seeds:
        if storage == "f64":
            rng = np.random.default_rng(seed)
            Ap, ATp = A, AT
            if entry_sd > 0.0:
                Ap, ATp = A.copy(), AT.copy()
                Ap.data = Ap.data + entry_sd * rng.standard_normal(Ap.nnz)
                ATp.data = ATp.data + entry_sd * rng.standard_normal(ATp.nnz)

            def vec(v):
                return np.asarray(v, np.float64)

            def pA(v, Ap=Ap):
                return (oracle.spmm(Ap, v) +
                        eps * rng.standard_normal((v.shape[0], A.shape[0])) * oracle.spmm(A, np.abs(v)))

            def pT(w, ATp=ATp):
                return (oracle.spmm(ATp, w) +
                        eps * rng.standard_normal((w.shape[0], AT.shape[0])) * oracle.spmm(AT, np.abs(w)))
        else:
            vec = f32
            fA, fT = Fp32Product(A, storage, 2 * seed + 1), Fp32Product(AT, storage, 2 * seed + 2)

            def operand(v):
                if storage == "f32":
                    return v
                m = _pow2_ceil(np.abs(v).max(axis=1))[:, None]
                return round_to(v / m, storage) * m

            def pA(v):
                return fA(operand(v))

            def pT(w):
                return fT(operand(w))
        ynorm = np.linalg.norm(vec(y), axis=1)
        x = np.zeros((B, xh_ref.shape[2]))
        r = vec(y)
        s = pT(r)
        p = s.copy()
        g = np.einsum("ij,ij->i", s, s)
        for k in range(iters):
            q = pA(p)
            d = np.einsum("ij,ij->i", q, q)
            ok = (g > 0) & (d > 0)
            a = vec(np.where(ok, g / np.where(ok, d, 1.0), 0.0))[:, None]
            r = vec(r - a * q)
            s = pT(r)
            gn = np.einsum("ij,ij->i", s, s)
            bt = np.where(ok, gn / np.where(g > 0, g, 1.0), 0.0)
            x = vec(x + a * p)
            p = vec(s + vec(bt)[:, None] * p)
            g = np.where(ok, gn, g)
            xr = xh_ref[k]
            dx = np.linalg.norm(x - xr, axis=1) / np.maximum(np.linalg.norm(xr, axis=1), 1e-300)
            res = np.linalg.norm(r, axis=1) / np.maximum(ynorm, 1e-300)
            dr = np.abs(res - res_ref[k + 1]) / np.maximum(res_ref[k + 1], 1e-300)
            env_x[k + 1] = np.maximum(env_x[k + 1], dx)
            env_r[k + 1] = np.maximum(env_r[k + 1], dr)
    return env_x, env_r
