"""Rounding envelope of CGLS iterates (test helper).

CGLS iterates are ill-conditioned under rounding: a relative perturbation of
size eps in every matrix product grows through the recurrences, and after
enough iterations the iterate differs from the exact one by far more than
eps.  This helper measures that growth with the FP64 oracle: it runs CGLS in
FP64 (the oracle's CSR products, numpy recurrences) with a seeded
multiplicative perturbation (1 + eps N(0,1)) on every element of every
product output, for several seeds at once, and returns per iteration k the
largest relative deviation of x_k and of the residual norm from the oracle's
unperturbed history.  A kernel that rounds at unit roundoff eps is expected
to deviate by about this much, not by less."""
import numpy as np

import oracle


def envelope_history(A, AT, y, xh_ref, res_ref, iters, eps, seeds=(0, 1, 2)):
    """y (B, rows); xh_ref (iters, B, cols): the oracle's x_1..x_iters;
    res_ref (iters+1, B): its residual history.  Returns (env_x, env_r), each
    (iters+1, B): max over seeds of ||x_k - x_k*|| / ||x_k*|| and of
    | r_k - r_k* | / r_k* (0 at k = 0, where both start from x = 0)."""
    y = np.asarray(y, np.float64)
    B, S = y.shape[0], len(seeds)
    rngs = [np.random.default_rng(s) for s in seeds]

    def pert(v):
        v = v.reshape(S, B, -1)
        for i, g in enumerate(rngs):
            v[i] *= 1.0 + eps * g.standard_normal(v[i].shape)
        return v.reshape(S * B, -1)

    Y = np.tile(y, (S, 1))
    ynorm = np.linalg.norm(Y, axis=1)
    x = np.zeros((S * B, A.shape[1]))
    r = Y.copy()
    s = pert(oracle.spmm(AT, r))
    p = s.copy()
    g = np.einsum("ij,ij->i", s, s)
    env_x = np.zeros((iters + 1, B))
    env_r = np.zeros((iters + 1, B))
    for k in range(iters):
        q = pert(oracle.spmm(A, p))
        d = np.einsum("ij,ij->i", q, q)
        ok = (g > 0) & (d > 0)
        a = np.where(ok, g / np.where(ok, d, 1.0), 0.0)
        x += a[:, None] * p
        r -= a[:, None] * q
        s = pert(oracle.spmm(AT, r))
        gn = np.einsum("ij,ij->i", s, s)
        bt = np.where(ok, gn / np.where(g > 0, g, 1.0), 0.0)
        p = s + bt[:, None] * p
        g = np.where(ok, gn, g)
        xr = xh_ref[k]
        dx = np.linalg.norm(x.reshape(S, B, -1) - xr[None], axis=2) / np.maximum(np.linalg.norm(xr, axis=1), 1e-300)
        res = (np.linalg.norm(r, axis=1) / np.maximum(ynorm, 1e-300)).reshape(S, B)
        dr = np.abs(res - res_ref[k + 1][None]) / np.maximum(res_ref[k + 1][None], 1e-300)
        env_x[k + 1] = dx.max(axis=0)
        env_r[k + 1] = dr.max(axis=0)
    return env_x, env_r
