"""Exact Newton directions for problems too large to form K densely (TEST
INFRASTRUCTURE ONLY).

Both use that the Schur complement of D in the doubly augmented matrix of
eq. (9) is the normal-equations matrix Q + B^T D^-1 B (Forsgren and Gill),
so (dx, dlam_A) solve
    (Q + B^T D^-1 B) dx = r1 + B^T D^-1 r2,   dlam_A = D^-1 (r2 - B dx).
`schur_direction` factors that n x n matrix densely (Cholesky).
`woodbury_direction` handles H = diag(h0) + U diag(wd) U^T with no general
rows: Q + B^T D^-1 B = diag(h0 + q_b) + V V^T with V = [U wd^1/2, C^T mu^-1/2],
inverted through the Woodbury identity with a (k+me) x (k+me) Cholesky.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .ipm import (Problem, State, Residuals, index_sets, reduced_system,
                  direction_from_solution, residuals)


def _B_ops(prob, S):
    me = prob.me

    def Bmul(v):
        return np.concatenate([prob.C @ v, S.AL @ v, -(S.AU @ v)])

    def BTmul(y):
        nl = S.L.size
        return prob.C.T @ y[:me] + S.AL.T @ y[me:me + nl] - S.AU.T @ y[me + nl:]
    return Bmul, BTmul


def schur_direction(prob: Problem, st: State, mu: float, res: Residuals = None):
    if res is None:
        res = residuals(prob, st, mu)
    S = index_sets(prob)
    _, _, D, r1, r2, qb = reduced_system(prob, st, res, mu, with_Q=False)
    me, nl = prob.me, S.L.size
    Dinv = 1.0 / D
    M = np.array(prob.Hdense(), dtype=np.float64)      # a fresh copy: factored in place
    M[np.diag_indices(prob.n)] += qb
    if me:
        M += prob.C.T @ (prob.C / mu)
    for blk, dsl in ((S.AL, slice(me, me + nl)), (S.AU, slice(me + nl, None))):
        if blk.shape[0]:
            if sp.issparse(blk):
                # B^T D^-1 B as a sparse product, added entry by entry
                T = (blk.T @ sp.diags(Dinv[dsl]) @ blk).tocoo()
                T.sum_duplicates()
                M[T.row, T.col] += T.data
            else:
                Bd = np.asarray(blk)
                M += Bd.T @ (Dinv[dsl][:, None] * Bd)
    Bmul, BTmul = _B_ops(prob, S)
    cf = sla.cho_factor(M, lower=True, overwrite_a=True)
    dx = sla.cho_solve(cf, r1 + BTmul(Dinv * r2))
    dlam = Dinv * (r2 - Bmul(dx))
    return direction_from_solution(prob, st, res, np.concatenate([dx, dlam]))


def woodbury_direction(prob: Problem, st: State, mu: float, res: Residuals = None,
                       h0=None, U=None, wd=None):
    if res is None:
        res = residuals(prob, st, mu)
    S = index_sets(prob)
    if S.L.size or S.U.size:
        raise ValueError("woodbury_direction needs a problem without general rows")
    _, _, D, r1, r2, qb = reduced_system(prob, st, res, mu, with_Q=False)
    delta = h0 + qb
    V = np.hstack([U * np.sqrt(wd), prob.C.T / np.sqrt(mu)])
    Dinv = 1.0 / D
    Bmul, BTmul = _B_ops(prob, S)
    g = r1 + BTmul(Dinv * r2)
    Vd = V / delta[:, None]
    small = np.eye(V.shape[1]) + V.T @ Vd
    cf = sla.cho_factor(small, lower=True)
    dx = g / delta - Vd @ sla.cho_solve(cf, Vd.T @ g)
    dlam = Dinv * (r2 - Bmul(dx))
    return direction_from_solution(prob, st, res, np.concatenate([dx, dlam]))
