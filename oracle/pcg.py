"""Textbook Jacobi-preconditioned conjugate gradients (TEST INFRASTRUCTURE
ONLY).

Section 3.1 (PCG with Jacobi preconditioning on the doubly augmented system)
and Section 5.1 (stop on the unpreconditioned residual, tolerance 1e-7, at
most 5000 iterations).  Reading: the tolerance is relative to ||rhs||_2, the
start is x0 = 0, and at the cap the current iterate is returned with a flag.
"""
from __future__ import annotations

import numpy as np


class PCGNotSPD(RuntimeError):
    pass


def pcg(Kmul, rhs: np.ndarray, diag: np.ndarray, tol: float = 1e-7,
        maxit: int = 5000):
    """Returns (x, iterations, converged, final relative residual)."""
    x = np.zeros_like(rhs)
    r = rhs.copy()
    nb = float(np.linalg.norm(rhs))
    if nb == 0.0:
        return x, 0, True, 0.0
    z = r / diag
    p = z.copy()
    rz = float(r @ z)
    for k in range(maxit):
        q = Kmul(p)
        pq = float(p @ q)
        if not pq > 0.0:
            raise PCGNotSPD(f"p^T K p = {pq} at iteration {k}")
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        rn = float(np.linalg.norm(r))
        if rn <= tol * nb:
            return x, k + 1, True, rn / nb
        z = r / diag
        rz_new = float(r @ z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, maxit, False, float(np.linalg.norm(r)) / nb
