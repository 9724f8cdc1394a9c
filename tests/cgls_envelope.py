"""Rounding envelope of CGLS iterates (test helper).

CGLS iterates are ill-conditioned under rounding: a relative perturbation of
size eps in every matrix product grows through the recurrences, and after
enough iterations the iterate differs from the exact one by far more than
eps.  This helper measures that growth with the FP64 oracle matrices: it runs
CGLS in FP64 (numpy, with the oracle's CSR A and A^T) several times with a
seeded multiplicative perturbation of size eps on every product output, and
returns the largest relative deviation of x_k from the oracle's unperturbed
iterate.  A kernel that rounds at unit roundoff eps is expected to deviate
by about this much, not by less."""
import numpy as np


def perturbed_cgls(A, AT, y, iters, eps, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros(A.shape[1])
    r = y.copy()
    s = AT @ r
    s = s * (1 + eps * rng.standard_normal(s.shape))
    p = s.copy()
    g = s @ s
    for _ in range(iters):
        q = A @ p
        q = q * (1 + eps * rng.standard_normal(q.shape))
        d = q @ q
        if g == 0.0 or d == 0.0:
            break
        a = g / d
        x = x + a * p
        r = r - a * q
        s = AT @ r
        s = s * (1 + eps * rng.standard_normal(s.shape))
        gn = s @ s
        p = s + (gn / g) * p
        g = gn
    return x


def envelope(A, AT, y, x_ref, iters, eps, seeds=(0, 1, 2)):
    """max over seeds of ||x_pert - x_ref|| / ||x_ref|| for each slice of y (B, rows)."""
    out = []
    for b in range(y.shape[0]):
        nref = np.linalg.norm(x_ref[b])
        dev = [np.linalg.norm(perturbed_cgls(A, AT, y[b], iters, eps, s) - x_ref[b]) / max(nref, 1e-300)
               for s in seeds]
        out.append(max(dev))
    return np.array(out)
