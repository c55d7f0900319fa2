"""Exact optimum of a tiny convex QP by active-set enumeration (TEST
INFRASTRUCTURE ONLY).  Independent of the interior point machinery: it pins
the whole IPM oracle on problems small enough to enumerate (eq. (1)).

Every inequality side is written g_i(x) = a_i^T x - beta_i >= 0; for each
subset of sides taken as equalities (together with C x = b) the KKT system
  [[H, -G_a^T, -C^T], [G_a, 0, 0], [C, 0, 0]] (x, nu, eta) = (-p, beta_a, b)
is solved; the optimum is the unique subset whose x is feasible and whose
inequality multipliers nu are nonnegative.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def _rows(prob):
    A = prob.A.toarray() if sp.issparse(prob.A) else np.asarray(prob.A)
    G, beta = [], []
    for i in range(A.shape[0]):
        if np.isfinite(prob.l[i]):
            G.append(A[i]); beta.append(prob.l[i])
        if np.isfinite(prob.u[i]):
            G.append(-A[i]); beta.append(-prob.u[i])
    I = np.eye(prob.n)
    for j in range(prob.n):
        if np.isfinite(prob.lx[j]):
            G.append(I[j]); beta.append(prob.lx[j])
        if np.isfinite(prob.ux[j]):
            G.append(-I[j]); beta.append(-prob.ux[j])
    return np.array(G).reshape(-1, prob.n), np.array(beta)


def brute_force_qp(prob, feas_tol: float = 1e-9, mult_tol: float = 1e-9):
    H = prob.Hdense()
    p = prob.p
    C, b = prob.C, prob.b
    G, beta = _rows(prob)
    n, me, mi = prob.n, C.shape[0], G.shape[0]
    best = None
    for k in range(0, min(mi, n) + 1):
        for act in itertools.combinations(range(mi), k):
            act = list(act)
            Ga = G[act]
            M = np.block([[H, -Ga.T, -C.T],
                          [Ga, np.zeros((k, k)), np.zeros((k, me))],
                          [C, np.zeros((me, k)), np.zeros((me, me))]])
            rhs = np.concatenate([-p, beta[act], b])
            try:
                sol = np.linalg.solve(M, rhs)
            except np.linalg.LinAlgError:
                continue
            x = sol[:n]
            nu = sol[n:n + k]
            if np.any(G @ x - beta < -feas_tol) or np.any(nu < -mult_tol):
                continue
            f = 0.5 * x @ H @ x + p @ x
            if best is None or f < best[1] - 1e-12:
                best = (x, f, act)
    if best is None:
        raise RuntimeError("no feasible active set")
    return best
