"""The unreduced Newton system of eq. (7), Section 3.1, formed densely and
solved by LU (TEST INFRASTRUCTURE ONLY).  It pins the block elimination that
leads to eqs. (8) and (9): both must give the same full direction.

Unknown order (as printed in eq. (7)):
  dx, dlam_lA, dlam_uA, dlam_lx, dlam_ux, dlam_e, ds_lA, ds_uA, ds_lx, ds_ux
Row order: r_H, r_e, r_lA, r_uA, r_lx, r_ux, r_c1, r_c2, r_c3, r_c4.
The lambda_e column of the first block row carries -C^T (reading of the
printed +C^T; see the module docstring of `ipm`).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .ipm import Direction, Problem, State, Residuals, index_sets


def _d(M):
    return M.toarray() if sp.issparse(M) else np.asarray(M)


def full_newton_matrix(prob: Problem, st: State, mu: float) -> np.ndarray:
    S = index_sets(prob)
    n, me = prob.n, prob.me
    nl, nu, nlx, nux = S.L.size, S.U.size, S.Lx.size, S.Ux.size
    AL, AU = _d(S.AL), _d(S.AU)
    Ilx = np.eye(n)[:, S.Lx]        # n x nlx, column j = e_{Lx[j]}
    Iux = np.eye(n)[:, S.Ux]
    sizes = [n, nl, nu, nlx, nux, me, nl, nu, nlx, nux]
    off = np.concatenate([[0], np.cumsum(sizes)])
    N = int(off[-1])
    J = np.zeros((N, N))

    def put(bi, bj, M):
        J[off[bi]:off[bi + 1], off[bj]:off[bj + 1]] = M

    # columns: 0 dx, 1 dlam_lA, 2 dlam_uA, 3 dlam_lx, 4 dlam_ux, 5 dlam_e,
    #          6 ds_lA, 7 ds_uA, 8 ds_lx, 9 ds_ux
    # rows reuse the same block sizes in the order r_H, r_e, r_lA, r_uA,
    # r_lx, r_ux, r_c1..r_c4; r_e has me rows, i.e. the size of block 5.
    rows = [n, me, nl, nu, nlx, nux, nl, nu, nlx, nux]
    roff = np.concatenate([[0], np.cumsum(rows)])

    def putr(ri, cj, M):
        J[roff[ri]:roff[ri + 1], off[cj]:off[cj + 1]] = M

    putr(0, 0, prob.Hdense())
    putr(0, 1, -AL.T)
    putr(0, 2, AU.T)
    putr(0, 3, -Ilx)
    putr(0, 4, Iux)
    putr(0, 5, -prob.C.T)
    putr(1, 0, prob.C)
    putr(1, 5, mu * np.eye(me))
    putr(2, 0, AL)
    putr(2, 6, -np.eye(nl))
    putr(3, 0, -AU)
    putr(3, 7, -np.eye(nu))
    putr(4, 0, Ilx.T)
    putr(4, 8, -np.eye(nlx))
    putr(5, 0, -Iux.T)
    putr(5, 9, -np.eye(nux))
    putr(6, 1, np.diag(st.s_lA))
    putr(6, 6, np.diag(st.lam_lA))
    putr(7, 2, np.diag(st.s_uA))
    putr(7, 7, np.diag(st.lam_uA))
    putr(8, 3, np.diag(st.s_lx))
    putr(8, 8, np.diag(st.lam_lx))
    putr(9, 4, np.diag(st.s_ux))
    putr(9, 9, np.diag(st.lam_ux))
    del put
    return J


def full_rhs(res: Residuals) -> np.ndarray:
    return -np.concatenate(res.blocks())


def full_newton_direction(prob: Problem, st: State, mu: float, res: Residuals) -> Direction:
    J = full_newton_matrix(prob, st, mu)
    z = np.linalg.solve(J, full_rhs(res))
    S = index_sets(prob)
    sizes = [prob.n, S.L.size, S.U.size, S.Lx.size, S.Ux.size, prob.me,
             S.L.size, S.U.size, S.Lx.size, S.Ux.size]
    parts = np.split(z, np.cumsum(sizes)[:-1])
    dx, dlA, duA, dlx, dux, de, slA, suA, slx, sux = parts
    return Direction(dx, de, dlA, duA, dlx, dux, slA, suA, slx, sux)
