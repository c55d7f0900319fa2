"""A Mehrotra predictor-corrector rule for the barrier parameter of
Algorithm 1 (TEST INFRASTRUCTURE ONLY; see the package docstring).

The paper's rule divides mu by ten whenever ||r|| < mu.  Section 5.2 finds
that rule too aggressive (the infeasibilities jump at every decrease), and
Section 7 leaves better mu updates to future work.  This is the classical
alternative (Mehrotra 1992), written on the same Newton systems (eq. (9),
through `newton_direction`) and the same state, ratio test and step:

  mu      = lam^T s / N_c at the current point (N_c finite sides), which is
            also the equality rows' penalty (D_e and r_e) for this iteration,
            so the two solves below share one matrix K;
  predictor: the Newton direction for complementarity target 0;
  its largest steps to the boundary (the ratio test with gamma = 1, capped
            at 1), alpha_x^a and alpha_lam^a;
  mu_aff  = (lam + alpha_lam^a dlam^a)^T (s + alpha_x^a ds^a) / N_c,
  sigma   = min(1, (mu_aff / mu)^3);
  corrector: the Newton direction for target tau = max(sigma mu, mu_stop / 2)
            with every complementarity row's residual increased by
            dlam^a * ds^a, i.e. lam ds + s dlam = tau - lam s - dlam^a ds^a;
  step:     the ratio test with gamma, as in Algorithm 1.

mu_stop = mu_tol / mu_div is the stopping accuracy below.  The target is
kept at or above half of it: left alone, sigma mu falls to 1e-13 within a
few iterations while the dual residual still sits at its rounding floor of a
few 1e-6, D = s / lam reaches 1e-17 and the doubly augmented matrix is no
longer positive definite in float64.

It stops when, at the new point, mu and the primal and dual residuals
(with that mu as the equality rows' penalty) are both below mu_tol / mu_div: the
accuracy at which the paper's rule stops (its last point has ||r(mu)|| < mu
with mu = mu_tol / mu_div).  Without inequality constraints there is no
complementarity to measure and the paper's rule is used.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from .ipm import (IPMOptions, IPMResult, Problem, Residuals, State, initial_point, newton_direction,
                  objective, residuals, solve, stacked_norm, step_lengths, take_step)

_PAIRS = (("lam_lA", "s_lA", "rc1"), ("lam_uA", "s_uA", "rc2"),
          ("lam_lx", "s_lx", "rc3"), ("lam_ux", "s_ux", "rc4"))
_DIR = {"lam_lA": ("dlam_lA", "ds_lA"), "lam_uA": ("dlam_uA", "ds_uA"),
        "lam_lx": ("dlam_lx", "ds_lx"), "lam_ux": ("dlam_ux", "ds_ux")}


def pair_count(st: State) -> int:
    return sum(getattr(st, lam).size for lam, _, _ in _PAIRS)


def complementarity(st: State, d=None, ax: float = 0.0, al: float = 0.0) -> float:
    """(lam + al dlam)^T (s + ax ds) over every inequality pair."""
    tot = 0.0
    for lam, s, _ in _PAIRS:
        lv, sv = getattr(st, lam), getattr(st, s)
        if d is not None:
            dl, ds = (getattr(d, k) for k in _DIR[lam])
            lv, sv = lv + al * dl, sv + ax * ds
        tot += float(lv @ sv)
    return tot


def target_residuals(prob: Problem, st: State, mu: float, tau: float, d_aff=None) -> Residuals:
    """The residuals of eq. (7) with penalty mu in the equality rows and
    complementarity target tau; with the predictor's direction d_aff, each
    complementarity residual also carries dlam^a * ds^a."""
    res = residuals(prob, st, mu)
    blocks = {}
    for lam, s, rc in _PAIRS:
        v = getattr(st, lam) * getattr(st, s) - tau
        if d_aff is not None:
            dl, ds = (getattr(d_aff, k) for k in _DIR[lam])
            v = v + dl * ds
        blocks[rc] = v
    return replace(res, **blocks)


def primal_dual_norm(res: Residuals) -> float:
    """||(r_H, r_e, r_lA, r_uA, r_lx, r_ux)||: the stack without complementarity."""
    return float(np.sqrt(sum(float(v @ v) for v in
                             (res.rH, res.re, res.rlA, res.ruA, res.rlx, res.rux))))


def solve_mpc(prob: Problem, opts: IPMOptions = IPMOptions(), direction=None,
              state: State = None) -> IPMResult:
    """Algorithm 1 with the predictor-corrector rule above.  `direction(prob,
    st, mu, res)` solves eq. (9) for the given residuals with penalty mu (the
    default is the dense Cholesky solve).  The log holds, per iteration, mu,
    sigma, the predictor's steps and the taken steps, and the residuals."""
    st = initial_point(prob) if state is None else state.copy()
    nc = pair_count(st)
    if nc == 0:
        return solve(prob, opts, direction=direction, state=st)
    if direction is None:
        direction = lambda pr, s, m, r: newton_direction(pr, s, m, r)[0]
    tol = opts.mu_tol / opts.mu_div
    log = []
    mu = complementarity(st) / nc
    for it in range(1, opts.max_iter + 1):
        d_aff = direction(prob, st, mu, target_residuals(prob, st, mu, 0.0))
        ax_a, al_a = step_lengths(st, d_aff, 1.0)
        mu_aff = complementarity(st, d_aff, ax_a, al_a) / nc
        sigma = min(1.0, (mu_aff / mu) ** 3)
        tau = max(sigma * mu, 0.5 * tol)
        d = direction(prob, st, mu, target_residuals(prob, st, mu, tau, d_aff))
        ax, al = step_lengths(st, d, opts.gamma)
        st = take_step(st, d, ax, al)
        mu_new = complementarity(st) / nc
        res_new = residuals(prob, st, mu_new)
        pd = primal_dual_norm(res_new)
        log.append(dict(it=it, mu=mu, sigma=sigma, tau=tau, alpha_x_aff=ax_a, alpha_lam_aff=al_a,
                        alpha_x=ax, alpha_lam=al, mu_new=mu_new, pd=pd,
                        rnorm=stacked_norm(res_new)))
        mu = mu_new
        if mu < tol and pd < tol:
            return IPMResult(st, mu, "converged", it, objective(prob, st.x), log)
    return IPMResult(st, mu, "max_iter", opts.max_iter, objective(prob, st.x), log)
