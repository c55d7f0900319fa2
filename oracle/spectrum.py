"""Spectrum of the doubly augmented matrix, with and without the Jacobi
preconditioner (TEST INFRASTRUCTURE ONLY).

Section 5.3 follows the condition number of the Newton systems along the
interior point iterations, for the matrix itself and for it preconditioned
by its diagonal.  This computes both from the definitions, densely: K of
eq. (9) at the state, its eigenvalues, and those of diag(K)^-1 K, which are
the eigenvalues of the symmetric matrix D^-1/2 K D^-1/2 with D = diag(K).
"""
from __future__ import annotations

import numpy as np

from .ipm import Problem, State, doubly_augmented, reduced_system, residuals


def kkt_dense(prob: Problem, st: State, mu: float) -> np.ndarray:
    """K of eq. (9) at (st, mu), dense."""
    res = residuals(prob, st, mu)
    Q, B, D, r1, r2, _ = reduced_system(prob, st, res, mu)
    K, _ = doubly_augmented(Q, B, D, r1, r2)
    return K


def jacobi_spectrum(prob: Problem, st: State, mu: float):
    """(smallest, largest) eigenvalue of diag(K)^-1 K."""
    K = kkt_dense(prob, st, mu)
    s = 1.0 / np.sqrt(np.diag(K))
    ev = np.linalg.eigvalsh(s[:, None] * K * s[None, :])
    return float(ev[0]), float(ev[-1])


def condition_numbers(prob: Problem, st: State, mu: float):
    """2-norm condition numbers of K and of diag(K)^-1 K (K is SPD)."""
    K = kkt_dense(prob, st, mu)
    ev = np.linalg.eigvalsh(K)
    lo, hi = jacobi_spectrum(prob, st, mu)
    return {"kappa": float(ev[-1] / ev[0]), "kappa_jacobi": hi / lo}
