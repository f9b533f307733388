"""Block-Jacobi preconditioned conjugate gradient (float64, CPU).

Appendix "Preconditioner": M is the block diagonal of H (the 3x3 diagonal block
of every free vertex, static + dynamic), inverted explicitly block by block.
The paper writes the solve in split form M^-1/2 H M^-1/2; in exact arithmetic
that is the same iteration as the standard left-preconditioned PCG below.

x0 = 0; stop when ||r||_2 <= rtol ||b||_2 (checked before each iteration) or
after max_iter iterations.  ``iters`` counts matrix-vector products.
"""
from __future__ import annotations

import numpy as np


def block_inverse(D):
    """Inverse of each 3x3 block of D (n, 3, 3)."""
    return np.linalg.inv(D)


def pcg(matvec, b, Minv, rtol=1e-8, max_iter=20000):
    """Solve H x = b.  matvec(v) returns H v for flat vectors of length 3n;
    Minv (n, 3, 3).  Returns (x, iters, rel_residual, status) with status
    'ok', 'noconv' or 'breakdown' (p^T H p <= 0)."""
    b = np.asarray(b, np.float64).ravel()
    n = Minv.shape[0]

    def prec(r):
        return np.einsum("vij,vj->vi", Minv, r.reshape(n, 3)).ravel()

    x = np.zeros_like(b)
    r = b.copy()
    bn = np.linalg.norm(b)
    z = prec(r)
    p = z.copy()
    rz = r @ z
    it = 0
    while np.linalg.norm(r) > rtol * bn:
        if it >= max_iter:
            return x, it, np.linalg.norm(r) / bn, "noconv"
        q = matvec(p)
        pq = p @ q
        if not pq > 0:
            return x, it, np.linalg.norm(r) / bn, "breakdown"
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        z = prec(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
    return x, it, (np.linalg.norm(r) / bn if bn > 0 else 0.0), "ok"
