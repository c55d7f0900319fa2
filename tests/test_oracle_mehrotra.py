"""Pins of the oracle's Mehrotra predictor-corrector rule (oracle.mehrotra),
the mu update that Sections 5.2 and 7 leave to future work: its two
directions against the rows of the unreduced Newton system (eq. (7)) that
define them, the predictor's scalars against a one-variable problem solved
by hand, and whole solves against brute-force optima and the paper's rule."""
import numpy as np
import pytest

import oracle as O
from oracle import mehrotra as M
from paper_2308_00637_amd import workloads as W
from tests.helpers import random_state

PAIRS = (("lam_lA", "s_lA", "dlam_lA", "ds_lA"), ("lam_uA", "s_uA", "dlam_uA", "ds_uA"),
         ("lam_lx", "s_lx", "dlam_lx", "ds_lx"), ("lam_ux", "s_ux", "dlam_ux", "ds_ux"))


def _general():
    return O.from_spec(W.random_bounded_qp(3, 12, 9, 2, 5, a_sparse=False))


def test_predictor_is_the_affine_scaling_direction():
    """Target 0: every complementarity row of eq. (7) reads
    lam ds + s dlam = -lam s, and the reduced solve equals the LU solve of
    the whole system."""
    prob = _general()
    st = random_state(prob, np.random.default_rng(5), 0.6)
    mu = 0.21
    res = M.target_residuals(prob, st, mu, 0.0)
    d = O.newton_direction(prob, st, mu, res)[0]
    full = O.full_newton_direction(prob, st, mu, res)
    for f in d.__dataclass_fields__:
        assert np.allclose(getattr(d, f), getattr(full, f), rtol=1e-9, atol=1e-11), f
    for lam, s, dl, ds in PAIRS:
        lv, sv = getattr(st, lam), getattr(st, s)
        lhs = lv * getattr(d, ds) + sv * getattr(d, dl)
        assert np.allclose(lhs, -lv * sv, rtol=1e-10, atol=1e-12), lam


def test_corrector_rows_carry_the_target_and_the_second_order_term():
    """Mehrotra's corrector: lam ds + s dlam = tau - lam s - dlam^a ds^a in
    every complementarity row, the other rows as in any Newton step (checked
    through the LU solve of eq. (7) with the same right-hand side)."""
    prob = _general()
    st = random_state(prob, np.random.default_rng(6), 0.6)
    mu, tau = 0.37, 0.05
    d_aff = O.newton_direction(prob, st, mu, M.target_residuals(prob, st, mu, 0.0))[0]
    res = M.target_residuals(prob, st, mu, tau, d_aff)
    d = O.newton_direction(prob, st, mu, res)[0]
    full = O.full_newton_direction(prob, st, mu, res)
    for f in d.__dataclass_fields__:
        assert np.allclose(getattr(d, f), getattr(full, f), rtol=1e-9, atol=1e-11), f
    for lam, s, dl, ds in PAIRS:
        lv, sv = getattr(st, lam), getattr(st, s)
        lhs = lv * getattr(d, ds) + sv * getattr(d, dl)
        rhs = tau - lv * sv - getattr(d_aff, dl) * getattr(d_aff, ds)
        assert np.allclose(lhs, rhs, rtol=1e-10, atol=1e-12), lam
    # the primal rows are the ordinary ones: A_L dx - ds_lA = -r_lA
    S = O.index_sets(prob)
    assert np.allclose(S.AL @ d.dx - d.ds_lA, -res.rlA, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("h, c, x, lam, s", [
    (2.0, 1.5, 0.8, 1.3, 0.6),    # the slack's step hits the boundary: alpha_x < 1, mu_aff = 0
    (1.0, 0.5, 0.5, 2.0, 0.5),    # full steps: mu_aff > 0, sigma = (mu_aff / mu)^3 = 0.0138
])
def test_predictor_scalars_on_one_variable_by_hand(h, c, x, lam, s):
    """min 1/2 h x^2 + c x, x >= 0, one pair (lam, s): the affine direction of
    the 3 x 3 system h dx - dlam = -r_H, dx - ds = -r_x, s dlam + lam ds = -lam s
    solved by hand, its steps to the boundary (gamma = 1), mu_aff and sigma."""
    spec = W.QPSpec(n=1, c=np.array([c]), h_kind="dense", H=np.array([[h]]),
                    lx=np.array([0.0]), ux=np.array([np.inf]))
    prob = O.from_spec(spec)
    e = np.zeros(0)
    st = O.State(x=np.array([x]), lam_e=e, lam_lA=e, lam_uA=e, lam_lx=np.array([lam]),
                 lam_ux=e, s_lA=e, s_uA=e, s_lx=np.array([s]), s_ux=e)
    rH, rx = h * x + c - lam, x - s
    dx = (-rH - lam - lam * rx / s) / (h + lam / s)
    ds = dx + rx
    dlam = -lam - lam * ds / s
    ax = min(1.0, -s / ds) if ds < 0 else 1.0
    al = min(1.0, -lam / dlam) if dlam < 0 else 1.0
    mu = lam * s
    mu_aff = (lam + al * dlam) * (s + ax * ds)
    sigma = min(1.0, (mu_aff / mu) ** 3)
    out = M.solve_mpc(prob, O.IPMOptions(max_iter=1), state=st)
    r = out.log[0]
    assert r["mu"] == pytest.approx(mu, rel=1e-15)
    assert r["alpha_x_aff"] == pytest.approx(ax, rel=1e-12)
    assert r["alpha_lam_aff"] == pytest.approx(al, rel=1e-12)
    assert r["sigma"] == pytest.approx(sigma, rel=1e-10)
    assert r["tau"] == pytest.approx(max(sigma * mu, 0.5e-7), rel=1e-10)


@pytest.mark.parametrize("seed", range(6))
def test_mpc_reaches_the_brute_force_optimum(seed):
    """Exact active-set optimum; the equality rows hold to mu |lam_e| under
    the penalty-barrier term, hence the tolerances of the paper-rule pin."""
    prob = O.from_spec(W.random_bounded_qp(seed, 5, 4, seed % 2, 3))
    x, f, act = O.brute_force_qp(prob)
    out = M.solve_mpc(prob)
    assert out.status == "converged"
    assert np.abs(out.state.x - x).max() < 1e-4
    assert abs(out.objective - f) <= 1e-5 * max(1.0, abs(f))


@pytest.mark.parametrize("name", ["tiny_dense", "rt_700x61", "qn_300"])
def test_mpc_matches_the_paper_rule_in_fewer_iterations(name):
    """Same optimum as the paper's rule (Algorithm 1), reached in fewer
    iterations, with mu and the primal and dual residuals below 1e-7."""
    spec = {"tiny_dense": W.tiny_dense, "rt_700x61": lambda: W.rt_qp(5, 700, 61, 0.08, 23, maxdose=0.6),
            "qn_300": lambda: W.qn_rt(6, 300, 12, 15)}[name]()
    prob = O.from_spec(spec)
    ref = O.solve(prob)
    out = M.solve_mpc(prob)
    print(f"{name}: paper rule {ref.iterations} iterations, Mehrotra {out.iterations}; "
          f"objectives {ref.objective:.12g} / {out.objective:.12g}")
    assert ref.status == "converged" and out.status == "converged"
    assert out.iterations < ref.iterations
    assert out.objective == pytest.approx(ref.objective, rel=1e-6)
    last = out.log[-1]
    assert last["mu_new"] < 1e-7 and last["pd"] < 1e-7
    res = O.residuals(prob, out.state, 0.0)
    assert M.primal_dual_norm(res) < 1e-7


def test_without_inequalities_the_paper_rule_runs():
    """No inequality pair: no complementarity to drive, so the paper's rule."""
    rng = np.random.default_rng(4)
    n = 5
    G = rng.standard_normal((n, n))
    spec = W.QPSpec(n=n, c=rng.standard_normal(n), h_kind="dense", H=G.T @ G + np.eye(n),
                    C=rng.standard_normal((2, n)), b=rng.standard_normal(2),
                    lx=np.full(n, -np.inf), ux=np.full(n, np.inf))
    prob = O.from_spec(spec)
    a, b = O.solve(prob), M.solve_mpc(prob)
    assert a.iterations == b.iterations and np.array_equal(a.state.x, b.state.x)
