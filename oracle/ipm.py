"""Primal-dual IPM of Section 3 of the paper, written out plainly (TEST
INFRASTRUCTURE ONLY; see the package docstring).

Notation follows Sections 2.1 and 3.1: objective 1/2 x^T H x + p^T x, general
rows l <= A x <= u, equality rows C x = b handled by the penalty-barrier term,
variable bounds lx <= x <= ux handled separately.  Only finite sides carry a
slack/multiplier pair, so every block here is compact: lam_lA and s_lA have one
entry per row with a finite lower side, and so on.

Readings of points the paper leaves open or prints inconsistently (each is
also listed in the design notes):
  * full Newton system, first block row: the lambda_e column carries -C^T (the
    residual r_H has -C^T lambda_e and the reduced form has -B^T with
    B = [C; A; -A]); the printed +C^T is taken as a typo.
  * r_uA = -A x - s_uA + u (the printed "+ s_u" contradicts the constraint
    -A x - s_u + u = 0 of the barrier problem).
  * r_c2 = lam_uA * s_uA - mu; r_lx, r_ux, r_c3, r_c4 by analogy for the
    variable bounds (the paper names them but does not print them).
  * Algorithm 1 says to solve the 2x2 augmented system by PCG; that system is
    unsymmetric, so the doubly augmented system (same solution) is solved.
  * Delta s comes from the primal rows and the bound Delta lambda from the
    complementarity rows of the full system (the paper does not say how the
    eliminated unknowns are recovered).
  * The ratio test ranges over all slacks (alpha_x) and all inequality
    multipliers (alpha_lambda); lambda_e is free, excluded from the ratio test
    but stepped with alpha_lambda.  An empty set gives a step of 1.
  * Initial point, mu0 = 1 and the iteration cap are not given; see
    `initial_point` and `IPMOptions`.
  * "||r|| < mu" uses the residuals at the new point with the current mu; after
    a decrease the next iteration's residuals use the new mu.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


class NotSPDError(RuntimeError):
    pass


# --------------------------------------------------------------------------
# Problem data (eq. (1), Section 2.1; variable bounds as in Section 3.1)
# --------------------------------------------------------------------------
@dataclass
class Problem:
    n: int
    Hmul: Callable[[np.ndarray], np.ndarray]
    Hdense: Callable[[], np.ndarray]
    Hdiag: Callable[[], np.ndarray]
    p: np.ndarray
    A: object            # dense ndarray or scipy sparse (m x n), may have 0 rows
    l: np.ndarray
    u: np.ndarray
    C: np.ndarray        # dense (me x n), may have 0 rows
    b: np.ndarray
    lx: np.ndarray
    ux: np.ndarray

    @property
    def m(self):
        return self.A.shape[0]

    @property
    def me(self):
        return self.C.shape[0]


def from_spec(spec) -> Problem:
    """Build the oracle's problem from a workload description (its own copy of
    every operator; nothing is shared with the GPU binding)."""
    n = spec.n
    if spec.h_kind == "dense":
        Hd = np.array(spec.H, dtype=np.float64)
        Hmul = lambda v: Hd @ v
        Hdense = lambda: Hd
        Hdiag = lambda: np.diag(Hd).copy()
        p = np.array(spec.c, dtype=np.float64)
    elif spec.h_kind == "lowrank":
        h0 = np.array(spec.h0, dtype=np.float64)
        U = np.array(spec.U, dtype=np.float64)
        wd = np.array(spec.wd, dtype=np.float64)
        Hmul = lambda v: h0 * v + U @ (wd * (U.T @ v))
        Hdense = lambda: np.diag(h0) + (U * wd) @ U.T
        Hdiag = lambda: h0 + (U * U) @ wd
        p = np.array(spec.c, dtype=np.float64)
    elif spec.h_kind == "ptwp":
        P = sp.csr_matrix(spec.P, dtype=np.float64)
        w = np.array(spec.w, dtype=np.float64)
        d = np.array(spec.d, dtype=np.float64)
        Hmul = lambda v: P.T @ (w * (P @ v))
        cache = {}

        def Hdense():
            # formed once per problem (a 20,000 x 20,000 P^T W P takes a minute)
            if "H" not in cache:
                cache["H"] = (P.T @ sp.diags(w) @ P).toarray()
            return cache["H"]
        Hdiag = lambda: np.asarray(P.multiply(P).T @ w).ravel()
        # 1/2 sum_v w_v (P_v x - d_v)^2 = 1/2 x^T P^T W P x - (P^T W d)^T x + const
        p = np.array(spec.c, dtype=np.float64) - P.T @ (w * d)
    else:
        raise ValueError(spec.h_kind)
    if spec.A is None:
        A = np.zeros((0, n))
        l = np.zeros(0)
        u = np.zeros(0)
    else:
        A = spec.A.astype(np.float64) if sp.issparse(spec.A) else np.array(spec.A, dtype=np.float64)
        l = np.array(spec.lA, dtype=np.float64)
        u = np.array(spec.uA, dtype=np.float64)
    C = np.zeros((0, n)) if spec.C is None else np.array(spec.C, dtype=np.float64)
    b = np.zeros(0) if spec.C is None else np.array(spec.b, dtype=np.float64)
    return Problem(n, Hmul, Hdense, Hdiag, p, A, l, u, C, b,
                   np.array(spec.lx, dtype=np.float64), np.array(spec.ux, dtype=np.float64))


@dataclass
class Sets:
    L: np.ndarray    # rows with finite lower side
    U: np.ndarray    # rows with finite upper side
    Lx: np.ndarray   # variables with finite lower bound
    Ux: np.ndarray   # variables with finite upper bound
    AL: object
    AU: object


def index_sets(prob: Problem) -> Sets:
    """Rows/variables that carry a slack-multiplier pair: only finite sides
    (the paper allows infinite sides without accounting for them explicitly)."""
    L = np.flatnonzero(np.isfinite(prob.l))
    U = np.flatnonzero(np.isfinite(prob.u))
    Lx = np.flatnonzero(np.isfinite(prob.lx))
    Ux = np.flatnonzero(np.isfinite(prob.ux))
    return Sets(L, U, Lx, Ux, prob.A[L], prob.A[U])


@dataclass
class State:
    x: np.ndarray
    lam_e: np.ndarray
    lam_lA: np.ndarray
    lam_uA: np.ndarray
    lam_lx: np.ndarray
    lam_ux: np.ndarray
    s_lA: np.ndarray
    s_uA: np.ndarray
    s_lx: np.ndarray
    s_ux: np.ndarray

    def copy(self) -> "State":
        return State(*(np.array(getattr(self, f)) for f in self.__dataclass_fields__))


def initial_point(prob: Problem) -> State:
    """Starting iterate (the paper gives none): x in the middle of two-sided
    bounds, one unit inside one-sided bounds, zero when free; bound slacks
    exact; row slacks max(distance, 1); all inequality multipliers 1, lam_e 0."""
    S = index_sets(prob)
    lx, ux = prob.lx, prob.ux
    x = np.zeros(prob.n)
    both = np.isfinite(lx) & np.isfinite(ux)
    lo = np.isfinite(lx) & ~np.isfinite(ux)
    hi = ~np.isfinite(lx) & np.isfinite(ux)
    x[both] = 0.5 * (lx[both] + ux[both])
    x[lo] = lx[lo] + 1.0
    x[hi] = ux[hi] - 1.0
    Ax_L = S.AL @ x
    Ax_U = S.AU @ x
    return State(
        x=x,
        lam_e=np.zeros(prob.me),
        lam_lA=np.ones(S.L.size), lam_uA=np.ones(S.U.size),
        lam_lx=np.ones(S.Lx.size), lam_ux=np.ones(S.Ux.size),
        s_lA=np.maximum(Ax_L - prob.l[S.L], 1.0),
        s_uA=np.maximum(prob.u[S.U] - Ax_U, 1.0),
        s_lx=x[S.Lx] - lx[S.Lx],
        s_ux=ux[S.Ux] - x[S.Ux])


# --------------------------------------------------------------------------
# Residuals: eq. (3) (perturbed KKT), extended to the variable bounds
# --------------------------------------------------------------------------
@dataclass
class Residuals:
    rH: np.ndarray
    re: np.ndarray
    rlA: np.ndarray
    ruA: np.ndarray
    rlx: np.ndarray
    rux: np.ndarray
    rc1: np.ndarray
    rc2: np.ndarray
    rc3: np.ndarray
    rc4: np.ndarray

    def blocks(self):
        return [self.rH, self.re, self.rlA, self.ruA, self.rlx, self.rux,
                self.rc1, self.rc2, self.rc3, self.rc4]


def _scatter(n, idx, v):
    out = np.zeros(n)
    out[idx] = v
    return out


def residuals(prob: Problem, st: State, mu: float) -> Residuals:
    """Right-hand side blocks of the full Newton system (eq. (7)), i.e. the
    perturbed optimality conditions (eq. (3)) with variable-bound rows."""
    S = index_sets(prob)
    n = prob.n
    rH = (prob.Hmul(st.x) + prob.p
          - S.AL.T @ st.lam_lA + S.AU.T @ st.lam_uA
          - _scatter(n, S.Lx, st.lam_lx) + _scatter(n, S.Ux, st.lam_ux)
          - prob.C.T @ st.lam_e)
    re = prob.C @ st.x - prob.b + mu * st.lam_e
    rlA = S.AL @ st.x - st.s_lA - prob.l[S.L]
    ruA = -(S.AU @ st.x) - st.s_uA + prob.u[S.U]
    rlx = st.x[S.Lx] - st.s_lx - prob.lx[S.Lx]
    rux = -st.x[S.Ux] - st.s_ux + prob.ux[S.Ux]
    rc1 = st.lam_lA * st.s_lA - mu
    rc2 = st.lam_uA * st.s_uA - mu
    rc3 = st.lam_lx * st.s_lx - mu
    rc4 = st.lam_ux * st.s_ux - mu
    return Residuals(rH, re, rlA, ruA, rlx, rux, rc1, rc2, rc3, rc4)


def stacked_norm(res: Residuals) -> float:
    """Euclidean norm of the whole residual stack (the ||r|| of Algorithm 1)."""
    return float(np.sqrt(sum(float(np.dot(v, v)) for v in res.blocks())))


def infeasibilities(res: Residuals):
    """Primal, dual and complementarity infeasibility as defined in Section 5.2."""
    primal = np.sqrt(sum(float(np.dot(v, v)) for v in (res.rlA, res.ruA, res.rlx, res.rux)))
    dual = float(np.linalg.norm(res.rH))
    compl = np.sqrt(sum(float(np.dot(v, v)) for v in (res.rc1, res.rc2, res.rc3, res.rc4)))
    return float(primal), dual, float(compl)


def objective(prob: Problem, x: np.ndarray) -> float:
    return float(0.5 * x @ prob.Hmul(x) + prob.p @ x)


# --------------------------------------------------------------------------
# Reduced and doubly augmented systems: eqs. (8) and (9), Section 3.1
# --------------------------------------------------------------------------
def _dense(M):
    return M.toarray() if sp.issparse(M) else np.asarray(M)


def reduced_system(prob: Problem, st: State, res: Residuals, mu: float,
                   with_Q: bool = True):
    """Q, B, D (diagonal, as a vector), r1, r2 of the 2x2 augmented system."""
    S = index_sets(prob)
    n = prob.n
    qb = _scatter(n, S.Lx, st.lam_lx / st.s_lx) + _scatter(n, S.Ux, st.lam_ux / st.s_ux)
    Q = prob.Hdense() + np.diag(qb) if with_Q else None
    B = np.vstack([prob.C, _dense(S.AL), -_dense(S.AU)]) if with_Q else None
    D = np.concatenate([np.full(prob.me, mu), st.s_lA / st.lam_lA, st.s_uA / st.lam_uA])
    r1 = (-res.rH
          - _scatter(n, S.Lx, res.rc3 / st.s_lx) + _scatter(n, S.Ux, res.rc4 / st.s_ux)
          - _scatter(n, S.Lx, st.lam_lx / st.s_lx * res.rlx)
          + _scatter(n, S.Ux, st.lam_ux / st.s_ux * res.rux))
    r2 = np.concatenate([-res.re,
                         -res.rlA - res.rc1 / st.lam_lA,
                         -res.ruA - res.rc2 / st.lam_uA])
    return Q, B, D, r1, r2, qb


def doubly_augmented(Q, B, D, r1, r2):
    """K = [[Q + 2 B^T D^-1 B, B^T], [B, D]] and its right-hand side (eq. (9))."""
    Dinv = 1.0 / D
    K = np.block([[Q + 2.0 * B.T @ (Dinv[:, None] * B), B.T],
                  [B, np.diag(D)]])
    rhs = np.concatenate([r1 + 2.0 * B.T @ (Dinv * r2), r2])
    return K, rhs


def newton_rhs_doubly(prob: Problem, st: State, mu: float):
    """Matrix-free right-hand side of eq. (9) at the current state; returns
    (rhs, residuals).  B^T y = C^T y_e + A_L^T y_l - A_U^T y_u."""
    S = index_sets(prob)
    res = residuals(prob, st, mu)
    _, _, D, r1, r2, _ = reduced_system(prob, st, res, mu, with_Q=False)
    me, nl = prob.me, S.L.size
    y = 2.0 * r2 / D
    BTy = prob.C.T @ y[:me] + S.AL.T @ y[me:me + nl] - S.AU.T @ y[me + nl:]
    return np.concatenate([r1 + BTy, r2]), res


def jacobi_diagonal(prob: Problem, st: State, mu: float) -> np.ndarray:
    """diag(K) of eq. (9), written from its definition: the top block is
    diag(Q) + 2 diag(B^T D^-1 B), the bottom block is D (Section 3.1)."""
    S = index_sets(prob)
    res = residuals(prob, st, mu)
    _, _, D, _, _, qb = reduced_system(prob, st, res, mu, with_Q=False)
    me, nl = prob.me, S.L.size
    Hd = prob.Hdiag()
    Dinv = 1.0 / D
    BtDB = np.zeros(prob.n)
    if me:
        BtDB += (prob.C * prob.C).T @ Dinv[:me]
    if nl:
        AL2 = S.AL.multiply(S.AL) if sp.issparse(S.AL) else S.AL * S.AL
        BtDB += AL2.T @ Dinv[me:me + nl]
    if S.U.size:
        AU2 = S.AU.multiply(S.AU) if sp.issparse(S.AU) else S.AU * S.AU
        BtDB += AU2.T @ Dinv[me + nl:]
    return np.concatenate([Hd + qb + 2.0 * BtDB, D])


def kkt_matvec(prob: Problem, st: State, mu: float, v: np.ndarray) -> np.ndarray:
    """K v for the doubly augmented K of eq. (9), without forming K (the
    matrix-free use of Section 3.2): t = B v_x; y_lam = t + D v_lam;
    y_x = Q v_x + B^T (2 D^-1 t + v_lam)."""
    S = index_sets(prob)
    n, me, nl = prob.n, prob.me, S.L.size
    res = residuals(prob, st, mu)
    _, _, D, _, _, qb = reduced_system(prob, st, res, mu, with_Q=False)
    vx, vl = v[:n], v[n:]
    t = np.concatenate([prob.C @ vx, S.AL @ vx, -(S.AU @ vx)])
    ylam = t + D * vl
    wv = 2.0 * t / D + vl
    BTw = prob.C.T @ wv[:me] + S.AL.T @ wv[me:me + nl] - S.AU.T @ wv[me + nl:]
    yx = prob.Hmul(vx) + qb * vx + BTw
    return np.concatenate([yx, ylam])


# --------------------------------------------------------------------------
# Newton direction (dense Cholesky of eq. (9)) and recovery of the rest
# --------------------------------------------------------------------------
@dataclass
class Direction:
    dx: np.ndarray
    dlam_e: np.ndarray
    dlam_lA: np.ndarray
    dlam_uA: np.ndarray
    dlam_lx: np.ndarray
    dlam_ux: np.ndarray
    ds_lA: np.ndarray
    ds_uA: np.ndarray
    ds_lx: np.ndarray
    ds_ux: np.ndarray


def direction_from_solution(prob: Problem, st: State, res: Residuals, sol: np.ndarray) -> Direction:
    """Unknowns eliminated in Section 3.1, recovered from (dx, dlam_A): slack
    steps from the primal rows of eq. (7), bound-multiplier steps from its
    complementarity rows."""
    S = index_sets(prob)
    n, me, nl = prob.n, prob.me, S.L.size
    dx = sol[:n]
    dlam = sol[n:]
    ds_lA = S.AL @ dx + res.rlA
    ds_uA = -(S.AU @ dx) + res.ruA
    ds_lx = dx[S.Lx] + res.rlx
    ds_ux = -dx[S.Ux] + res.rux
    dlam_lx = -(res.rc3 + st.lam_lx * ds_lx) / st.s_lx
    dlam_ux = -(res.rc4 + st.lam_ux * ds_ux) / st.s_ux
    return Direction(dx, dlam[:me], dlam[me:me + nl], dlam[me + nl:],
                     dlam_lx, dlam_ux, ds_lA, ds_uA, ds_lx, ds_ux)


def newton_direction(prob: Problem, st: State, mu: float, res: Optional[Residuals] = None):
    """Form K densely and solve eq. (9) by Cholesky."""
    if res is None:
        res = residuals(prob, st, mu)
    Q, B, D, r1, r2, _ = reduced_system(prob, st, res, mu)
    K, rhs = doubly_augmented(Q, B, D, r1, r2)
    try:
        cf = sla.cho_factor(K, lower=True, check_finite=True)
    except np.linalg.LinAlgError as e:
        raise NotSPDError(str(e))
    sol = sla.cho_solve(cf, rhs)
    return direction_from_solution(prob, st, res, sol), sol, rhs


def step_lengths(st: State, d: Direction, gamma: float = 0.99):
    """Ratio test of eq. (10)."""
    def ratio(vals, steps):
        v = np.concatenate(vals)
        dv = np.concatenate(steps)
        neg = dv < 0
        if not np.any(neg):
            return 1.0
        return float(min(1.0, gamma * np.min(-v[neg] / dv[neg])))
    ax = ratio([st.s_lA, st.s_uA, st.s_lx, st.s_ux], [d.ds_lA, d.ds_uA, d.ds_lx, d.ds_ux])
    al = ratio([st.lam_lA, st.lam_uA, st.lam_lx, st.lam_ux],
               [d.dlam_lA, d.dlam_uA, d.dlam_lx, d.dlam_ux])
    return ax, al


def take_step(st: State, d: Direction, ax: float, al: float) -> State:
    """x and s move by alpha_x, every multiplier by alpha_lambda (Algorithm 1)."""
    return State(
        x=st.x + ax * d.dx,
        lam_e=st.lam_e + al * d.dlam_e,
        lam_lA=st.lam_lA + al * d.dlam_lA, lam_uA=st.lam_uA + al * d.dlam_uA,
        lam_lx=st.lam_lx + al * d.dlam_lx, lam_ux=st.lam_ux + al * d.dlam_ux,
        s_lA=st.s_lA + ax * d.ds_lA, s_uA=st.s_uA + ax * d.ds_uA,
        s_lx=st.s_lx + ax * d.ds_lx, s_ux=st.s_ux + ax * d.ds_ux)


# --------------------------------------------------------------------------
# Algorithm 1
# --------------------------------------------------------------------------
@dataclass
class IPMOptions:
    gamma: float = 0.99
    mu0: float = 1.0
    mu_tol: float = 1e-6
    mu_div: float = 10.0
    max_iter: int = 200


@dataclass
class IPMResult:
    state: State
    mu: float
    status: str
    iterations: int
    objective: float
    log: list = field(default_factory=list)


def solve(prob: Problem, opts: IPMOptions = IPMOptions(), direction=None,
          state: Optional[State] = None) -> IPMResult:
    """Algorithm 1.  `direction(prob, st, mu, res)` returns a Direction; the
    default is the dense Cholesky solve of eq. (9)."""
    if direction is None:
        direction = lambda pr, s, m, r: newton_direction(pr, s, m, r)[0]
    st = initial_point(prob) if state is None else state.copy()
    mu = opts.mu0
    log = []
    for it in range(1, opts.max_iter + 1):
        res = residuals(prob, st, mu)
        d = direction(prob, st, mu, res)
        ax, al = step_lengths(st, d, opts.gamma)
        st = take_step(st, d, ax, al)
        res = residuals(prob, st, mu)
        nr = stacked_norm(res)
        pr, du, co = infeasibilities(res)
        log.append(dict(it=it, mu=mu, rnorm=nr, alpha_x=ax, alpha_lam=al,
                        primal=pr, dual=du, compl=co))
        if nr < mu:
            if mu < opts.mu_tol:
                return IPMResult(st, mu, "converged", it, objective(prob, st.x), log)
            mu = mu / opts.mu_div
    return IPMResult(st, mu, "max_iter", opts.max_iter, objective(prob, st.x), log)
