"""Spectrum and condition numbers of the doubly augmented matrix, with and
without the Jacobi preconditioner (TEST INFRASTRUCTURE ONLY).

Section 5.3 follows the condition number of the Newton systems along the
interior point iterations, for the matrix itself and for it preconditioned
by its diagonal, with a 1-norm condition estimator.  This computes both from
the definitions, densely: K of eq. (9) at the state, its eigenvalues, and
those of diag(K)^-1 K, which are the eigenvalues of the symmetric matrix
D^-1/2 K D^-1/2 with D = diag(K); and the 1-norm estimates of Hager's method
as refined by Higham, with solves through a Cholesky factor of K.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

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


def onenorm_inverse_estimate(solve, solve_t, n: int, maxiter: int = 5) -> float:
    """Lower estimate of ||A^-1||_1 from products with A^-1 and A^-T: Hager's
    method (1984), a steepest ascent of ||A^-1 x||_1 over the unit 1-norm
    ball that moves between its vertices, with Higham's (1988) safeguards:
    stop when the estimate no longer grows or the gradient's largest entry
    is the current vertex's, keep the largest value seen, and compare it with
    the estimate from the alternating vector x_i = (-1)^i (1 + i/(n-1)).
    Every value it returns is ||A^-1 x||_1 / ||x||_1 for some x, so it never
    exceeds the true norm."""
    x = np.full(n, 1.0 / n)
    est = 0.0
    for k in range(maxiter):
        y = solve(x)
        new = float(np.abs(y).sum())
        if k > 0 and new <= est:
            break
        est = new
        xi = np.where(y >= 0, 1.0, -1.0)
        z = solve_t(xi)
        j = int(np.argmax(np.abs(z)))
        if k > 0 and abs(z[j]) <= z @ x:
            break
        x = np.zeros(n)
        x[j] = 1.0
    i = np.arange(n)
    alt = np.where(i % 2 == 0, 1.0, -1.0) * (1.0 + i / max(n - 1, 1))
    return max(est, 2.0 * float(np.abs(solve(alt)).sum()) / (3.0 * n))


def condest(prob: Problem, st: State, mu: float):
    """1-norm condition estimates (Section 5.3) of K and of the Jacobi
    preconditioned matrix, each ||M||_1 times the estimate of ||M^-1||_1 with
    the solves through a Cholesky factor of M.  The preconditioned matrix is
    taken in its symmetric form D^-1/2 K D^-1/2, D = diag(K): it is the one a
    Cholesky factorisation applies to, and it has the spectrum of diag(K)^-1 K
    that preconditioned CG sees."""
    K = kkt_dense(prob, st, mu)
    s = 1.0 / np.sqrt(np.diag(K))
    out = {}
    for key, M in (("kappa1", K), ("kappa1_jacobi", s[:, None] * K * s[None, :])):
        cf = sla.cho_factor(M, lower=True)
        solve = lambda v, cf=cf: sla.cho_solve(cf, v)
        out[key] = float(np.abs(M).sum(axis=0).max()) * onenorm_inverse_estimate(
            solve, solve, M.shape[0])
    return out


def condest_path(prob: Problem, direction=None, opts=None):
    """The condition estimates of Section 5.3 along the interior point path:
    runs Algorithm 1 (`ipm.solve`, with `direction` as there) and evaluates
    `condest` on every Newton system before its solve.  Returns the result
    and one row per Newton system: it, mu, kappa1, kappa1_jacobi and the
    state the system is formed at."""
    from .ipm import IPMOptions, newton_direction, solve
    if direction is None:
        direction = lambda pr, s, m, r: newton_direction(pr, s, m, r)[0]
    rows = []

    def record(pr, st, mu, res):
        rows.append(dict(it=len(rows) + 1, mu=mu, state=st.copy(), **condest(pr, st, mu)))
        return direction(pr, st, mu, res)

    result = solve(prob, IPMOptions() if opts is None else opts, direction=record)
    return result, rows
