"""Adjoint sensitivities of the IPM solution (TEST INFRASTRUCTURE ONLY).

Not part of the paper: this is the implicit-function derivative of the
perturbed optimality conditions (eq. (3), with the variable-bound rows of
eq. (7)) at a fixed barrier parameter mu.  With F(z; theta) = 0 at the returned
point and J = dF/dz (the matrix of eq. (7)),
    dL/dtheta = -xi^T dF/dtheta,   J^T xi = dL/dz.
Here J^T is formed densely and solved by LU, with no use of the reduced or
doubly augmented forms, so it checks any reduction independently.

Parameter derivatives of F:
  r_H = Hx + p - ...   ->  dF/dp   = I on the r_H rows
  r_lA = A_L x - s - l ->  dF/dl_L = -I on the r_lA rows
  r_uA = -A_U x - s + u -> dF/du_U = +I on the r_uA rows
  r_e = Cx - b + mu lam_e -> dF/db = -I on the r_e rows
  ptwp: H = P^T W P and p = c - P^T W d, so dr_H/dw_v = P_v^T (P_v x - d_v).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fullsystem import full_newton_matrix, full_newton_direction
from .ipm import Problem, State, index_sets, residuals, stacked_norm, take_step


def adjoint_gradients(prob: Problem, st: State, mu: float, grad_x: np.ndarray,
                      P=None, w=None, d=None):
    S = index_sets(prob)
    n, me, nl, nu = prob.n, prob.me, S.L.size, S.U.size
    J = full_newton_matrix(prob, st, mu)
    g = np.zeros(J.shape[0])
    g[:n] = grad_x
    xi = np.linalg.solve(J.T, g)
    xi_H = xi[:n]
    xi_e = xi[n:n + me]
    xi_lA = xi[n + me:n + me + nl]
    xi_uA = xi[n + me + nl:n + me + nl + nu]
    out = {
        "c": -xi_H,
        "l": np.zeros(prob.m), "u": np.zeros(prob.m),
        "b": xi_e.copy(),
        "xi_H": xi_H,
    }
    out["l"][S.L] = xi_lA
    out["u"][S.U] = -xi_uA
    if P is not None:
        P = sp.csr_matrix(P)
        out["w"] = -(P @ xi_H) * (P @ st.x - d)
    return out


def _max_step(vals, steps):
    """Full step when it keeps every entry positive, else 0.99 of the way to
    the boundary."""
    v = np.concatenate(vals)
    dv = np.concatenate(steps)
    neg = dv < 0
    if not np.any(neg):
        return 1.0
    r = float(np.min(-v[neg] / dv[neg]))
    return 1.0 if r > 1.0 else 0.99 * r


def center(prob: Problem, st: State, mu: float, tol: float = 1e-13,
           max_iter: int = 60) -> State:
    """Newton's method on F_mu(z) = 0 at fixed mu with exact (LU) steps of
    eq. (7), kept strictly interior by the ratio test of eq. (10)."""
    st = st.copy()
    for _ in range(max_iter):
        res = residuals(prob, st, mu)
        if stacked_norm(res) <= tol:
            return st
        d = full_newton_direction(prob, st, mu, res)
        ax = _max_step([st.s_lA, st.s_uA, st.s_lx, st.s_ux],
                       [d.ds_lA, d.ds_uA, d.ds_lx, d.ds_ux])
        al = _max_step([st.lam_lA, st.lam_uA, st.lam_lx, st.lam_ux],
                       [d.dlam_lA, d.dlam_uA, d.dlam_lx, d.dlam_ux])
        st = take_step(st, d, ax, al)
    res = residuals(prob, st, mu)
    if stacked_norm(res) > 1e3 * tol:
        raise RuntimeError(f"centering stalled at {stacked_norm(res)}")
    return st
