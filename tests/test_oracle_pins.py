"""Pins of the CPU oracle against facts fixed by the paper and by mathematics,
not by the oracle itself.  CPU only.

Each test names what a plausible mistake in the oracle would break.
"""
import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

import oracle as O
from oracle.pcg import pcg
from paper_2308_00637_amd import workloads as W
from tests.helpers import random_state, rel


def general(seed, n=7, m=6, me=2, mg=4, a_sparse=False, h_kind="dense"):
    return O.from_spec(W.random_bounded_qp(seed, n, m, me, mg, a_sparse=a_sparse,
                                           h_kind=h_kind))


# ---------------------------------------------------------------- residuals
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_residuals_vanish_at_barrier_stationary_point(seed):
    """Build data so that (x, lam, s) is a stationary point of the barrier
    problem of eq. (2): the constraint rows fix l, u, lx, ux, b from x and s;
    lam * s = mu comes from d/ds of -mu log s; p from d/dx of the Lagrangian.
    Every residual block of eq. (3) must then vanish.  A wrong sign in any
    block breaks this."""
    rng = np.random.default_rng(seed)
    n, m, me, mu = 6, 5, 2, 0.3
    spec = W.random_bounded_qp(seed, n, m, me, 3)
    prob = O.from_spec(spec)
    S = O.index_sets(prob)
    x = rng.standard_normal(n)
    s_lA, s_uA = rng.uniform(0.5, 2, S.L.size), rng.uniform(0.5, 2, S.U.size)
    s_lx, s_ux = rng.uniform(0.5, 2, S.Lx.size), rng.uniform(0.5, 2, S.Ux.size)
    lam_lA, lam_uA, lam_lx, lam_ux = mu / s_lA, mu / s_uA, mu / s_lx, mu / s_ux
    lam_e = rng.standard_normal(me)
    A = prob.A
    prob.l = np.full(m, -np.inf); prob.u = np.full(m, np.inf)
    prob.l[S.L] = A[S.L] @ x - s_lA           # A x - s_l - l = 0
    prob.u[S.U] = A[S.U] @ x + s_uA           # -A x - s_u + u = 0
    prob.lx = np.full(n, -np.inf); prob.ux = np.full(n, np.inf)
    prob.lx[S.Lx] = x[S.Lx] - s_lx
    prob.ux[S.Ux] = x[S.Ux] + s_ux
    # penalty term (1/2mu)||Cx-b||^2 with lam_e = -(Cx - b)/mu
    prob.b = prob.C @ x + mu * lam_e
    # Lagrangian gradient: Hx + p + C^T(Cx-b)/mu - A^T lam_l + A^T lam_u - lam_lx + lam_ux = 0
    g = np.zeros(n)
    g += -A[S.L].T @ lam_lA + A[S.U].T @ lam_uA
    g[S.Lx] -= lam_lx
    g[S.Ux] += lam_ux
    prob.p = -(prob.Hmul(x) + prob.C.T @ (-lam_e) + g)
    st = O.State(x, lam_e, lam_lA, lam_uA, lam_lx, lam_ux, s_lA, s_uA, s_lx, s_ux)
    res = O.residuals(prob, st, mu)
    assert O.stacked_norm(res) < 1e-12
    d, sol, rhs = O.newton_direction(prob, st, mu)
    assert np.abs(rhs).max() < 1e-12 and np.abs(sol).max() < 1e-10


# ------------------------------------------------- eliminations (P2, P3, P1)
@pytest.mark.parametrize("seed,sparse_a", [(0, False), (1, True), (2, False), (3, True)])
def test_doubly_augmented_matches_full_newton_system(seed, sparse_a):
    """The 10-block system of eq. (7), solved by LU, and the Cholesky solve of
    eq. (9) followed by recovery give the same full direction at an arbitrary
    interior state (pins every sign of eqs. (8)-(9) and of the recovery)."""
    rng = np.random.default_rng(100 + seed)
    prob = general(seed, a_sparse=sparse_a)
    st = random_state(prob, rng, spread=0.5)
    mu = 0.7
    res = O.residuals(prob, st, mu)
    d1, _, _ = O.newton_direction(prob, st, mu, res)
    d2 = O.full_newton_direction(prob, st, mu, res)
    for f in d1.__dataclass_fields__:
        a, b = getattr(d1, f), getattr(d2, f)
        assert np.allclose(a, b, rtol=1e-9, atol=1e-9 * max(1, np.abs(b).max(initial=0))), f


def test_schur_complement_direction_matches():
    """(Q + B^T D^-1 B) dx = r1 + B^T D^-1 r2 is the Schur complement of D in K."""
    rng = np.random.default_rng(7)
    prob = general(4)
    st = random_state(prob, rng)
    d1, _, _ = O.newton_direction(prob, st, 0.2)
    d2 = O.schur_direction(prob, st, 0.2)
    assert rel(d2.dx, d1.dx) < 1e-10
    assert rel(d2.dlam_lA, d1.dlam_lA) < 1e-9


def test_kkt_is_spd_along_the_iterates():
    """Eq. (9) is SPD for convex QPs (Section 3.1): at every iterate."""
    prob = general(5)
    st = O.initial_point(prob)
    mu = 1.0
    for _ in range(12):
        res = O.residuals(prob, st, mu)
        Q, B, D, r1, r2, _ = O.reduced_system(prob, st, res, mu)
        K, _ = O.doubly_augmented(Q, B, D, r1, r2)
        assert np.allclose(K, K.T)
        assert np.linalg.eigvalsh(K).min() > 0
        d, _, _ = O.newton_direction(prob, st, mu, res)
        ax, al = O.step_lengths(st, d)
        st = O.take_step(st, d, ax, al)
        mu *= 0.5


# ----------------------------------------------- operator, Jacobi (P4, P5)
@pytest.mark.parametrize("h_kind", ["dense", "lowrank", "ptwp"])
def test_matrix_free_operator_and_jacobi(h_kind):
    rng = np.random.default_rng(11)
    if h_kind == "ptwp":
        prob = O.from_spec(W.rt_qp(8, 90, 12, 0.2, 7, maxdose=0.5))
    else:
        prob = general(6, a_sparse=True, h_kind=h_kind)
    st = random_state(prob, rng)
    mu = 0.3
    res = O.residuals(prob, st, mu)
    Q, B, D, r1, r2, _ = O.reduced_system(prob, st, res, mu)
    K, rhs = O.doubly_augmented(Q, B, D, r1, r2)
    N = K.shape[0]
    cols = np.stack([O.kkt_matvec(prob, st, mu, e) for e in np.eye(N)], axis=1)
    assert np.allclose(cols, K, rtol=1e-12, atol=1e-12 * np.abs(K).max())
    assert np.allclose(O.jacobi_diagonal(prob, st, mu), np.diag(K), rtol=1e-12)
    rhs2, _ = O.newton_rhs_doubly(prob, st, mu)
    assert np.allclose(rhs2, rhs, rtol=1e-12, atol=1e-12 * np.abs(rhs).max())
    u, v = rng.standard_normal(N), rng.standard_normal(N)
    Ku, Kv = O.kkt_matvec(prob, st, mu, u), O.kkt_matvec(prob, st, mu, v)
    assert abs(u @ Kv - v @ Ku) < 1e-11 * abs(u @ Kv)
    assert v @ Kv > 0


def test_pcg_agrees_with_cholesky():
    """Jacobi PCG at tolerance 1e-7 (Section 5.1) reproduces the direct solve to
    within the residual bound kappa(K) * tol."""
    rng = np.random.default_rng(3)
    prob = general(7, n=30, m=25, me=2, mg=10)
    st = random_state(prob, rng, 0.7)
    mu = 0.05
    res = O.residuals(prob, st, mu)
    Q, B, D, r1, r2, _ = O.reduced_system(prob, st, res, mu)
    K, rhs = O.doubly_augmented(Q, B, D, r1, r2)
    dg = np.diag(K)
    x, it, conv, rr = pcg(lambda v: K @ v, rhs, dg, 1e-10, 5000)
    assert conv and rr <= 1e-10
    xd = np.linalg.solve(K, rhs)
    Kj = K / np.sqrt(np.outer(dg, dg))
    kappa = np.linalg.cond(Kj)
    assert rel(x, xd) <= 10 * kappa * 1e-10


# ------------------------------------------------------- IPM invariants (P7)
def test_primal_residual_contracts_by_one_minus_alpha():
    """Slack steps come from the primal rows, so each primal residual block
    scales by exactly (1 - alpha_x) per step (to rounding)."""
    prob = general(8)
    st = O.initial_point(prob)
    mu = 1.0
    for _ in range(6):
        res = O.residuals(prob, st, mu)
        d, _, _ = O.newton_direction(prob, st, mu, res)
        ax, al = O.step_lengths(st, d)
        st = O.take_step(st, d, ax, al)
        res2 = O.residuals(prob, st, mu)
        for a, b in ((res.rlA, res2.rlA), (res.ruA, res2.ruA), (res.rlx, res2.rlx), (res.rux, res2.rux)):
            assert np.allclose(b, (1 - ax) * a, atol=1e-12 * (1 + np.abs(a).max(initial=0)))


def test_ratio_test_reaches_fraction_of_boundary():
    """Eq. (10): when alpha < 1 the step reaches exactly gamma of the way to the
    nearest zero; all entries stay positive."""
    rng = np.random.default_rng(9)
    prob = general(9)
    for _ in range(5):
        st = random_state(prob, rng)
        d, _, _ = O.newton_direction(prob, st, 0.5)
        ax, al = O.step_lengths(st, d, 0.99)
        s = np.concatenate([st.s_lA, st.s_uA, st.s_lx, st.s_ux])
        ds = np.concatenate([d.ds_lA, d.ds_uA, d.ds_lx, d.ds_ux])
        assert np.all(s + ax * ds > 0)
        if ax < 1:
            assert abs(np.min(s + (ax / 0.99) * ds)) < 1e-12 * np.abs(s).max()
        lam = np.concatenate([st.lam_lA, st.lam_uA, st.lam_lx, st.lam_ux])
        dl = np.concatenate([d.dlam_lA, d.dlam_uA, d.dlam_lx, d.dlam_ux])
        assert np.all(lam + al * dl > 0)
        if al < 1:
            assert abs(np.min(lam + (al / 0.99) * dl)) < 1e-12 * np.abs(lam).max()


# ------------------------------------------------- closed forms (P8, P9, P10)
def test_unconstrained_closed_form_and_iteration_count():
    """No constraints: the first Newton step lands on x = -H^-1 p, and the
    mu schedule 1 -> 1e-7 by repeated FP64 division ends after exactly 8
    iterations (mu6 = 1.0000000000000002e-06 is not below 1e-6)."""
    rng = np.random.default_rng(0)
    n = 8
    G = rng.standard_normal((n, n))
    spec = W.QPSpec(n=n, c=rng.standard_normal(n), h_kind="dense", H=G.T @ G + np.eye(n))
    prob = O.from_spec(spec)
    r = O.solve(prob)
    assert r.status == "converged" and r.iterations == 8
    assert np.allclose(r.state.x, -np.linalg.solve(spec.H, spec.c), rtol=1e-12)
    mus = [e["mu"] for e in r.log]
    assert mus[0] == 1.0 and mus[6] == 1.0000000000000002e-06 and mus[7] < 1e-6


def test_box_only_separable_closed_form():
    rng = np.random.default_rng(1)
    n = 12
    h = rng.uniform(0.5, 2, n)
    c = rng.standard_normal(n) * 3
    lx, ux = -np.ones(n), np.ones(n)
    prob = O.from_spec(W.QPSpec(n=n, c=c, h_kind="dense", H=np.diag(h), lx=lx, ux=ux))
    r = O.solve(prob)
    assert r.status == "converged"
    assert np.abs(r.state.x - np.clip(-c / h, lx, ux)).max() < 1e-5


def test_equality_only_penalty_closed_form():
    """Only C x = b: the penalty-barrier system is linear, so one Newton step
    solves (H + C^T C / mu) x = -p + C^T b / mu at mu = 1; as mu -> 0 the
    iterate tends to the solution of the equality-constrained QP."""
    rng = np.random.default_rng(2)
    n, me = 9, 3
    G = rng.standard_normal((n, n))
    H = G.T @ G + np.eye(n)
    c = rng.standard_normal(n)
    C = rng.standard_normal((me, n))
    b = rng.standard_normal(me)
    prob = O.from_spec(W.QPSpec(n=n, c=c, h_kind="dense", H=H, C=C, b=b))
    r = O.solve(prob, O.IPMOptions(max_iter=1))
    x1 = np.linalg.solve(H + C.T @ C / 1.0, -c + C.T @ b / 1.0)
    assert np.allclose(r.state.x, x1, rtol=1e-10)
    r = O.solve(prob)
    kkt = np.linalg.solve(np.block([[H, C.T], [C, np.zeros((me, me))]]), np.concatenate([-c, b]))
    assert np.abs(r.state.x - kkt[:n]).max() < 1e-5


# ---------------------------------------------- whole-oracle pins (P11, P12)
@pytest.mark.parametrize("seed", range(6))
def test_ipm_matches_brute_force_active_set(seed):
    spec = W.random_bounded_qp(seed, 5, 4, seed % 2, 3)
    prob = O.from_spec(spec)
    r = O.solve(prob)
    assert r.status == "converged"
    x, f, act = O.brute_force_qp(prob)
    assert np.abs(r.state.x - x).max() < 1e-4
    assert abs(r.objective - f) <= 1e-5 * max(1.0, abs(f))


def test_ipm_matches_scipy_trust_constr():
    spec = W.random_bounded_qp(21, 10, 8, 2, 5)
    prob = O.from_spec(spec)
    r = O.solve(prob)
    H = prob.Hdense()
    cons = [so.LinearConstraint(prob.A, prob.l, prob.u),
            so.LinearConstraint(prob.C, prob.b, prob.b)]
    sol = so.minimize(lambda x: 0.5 * x @ H @ x + prob.p @ x, np.zeros(prob.n),
                      jac=lambda x: H @ x + prob.p, hess=lambda x: H,
                      method="trust-constr", constraints=cons,
                      bounds=so.Bounds(prob.lx, prob.ux),
                      options=dict(gtol=1e-10, xtol=1e-12, maxiter=5000))
    assert abs(r.objective - sol.fun) < 1e-4 * max(1, abs(sol.fun))
    assert np.abs(r.state.x - sol.x).max() < 1e-3


def test_initial_point_is_strictly_interior():
    prob = general(12)
    st = O.initial_point(prob)
    for f in ("lam_lA", "lam_uA", "lam_lx", "lam_ux", "s_lA", "s_uA", "s_lx", "s_ux"):
        assert np.all(getattr(st, f) > 0)
    res = O.residuals(prob, st, 1.0)
    assert np.allclose(res.rlx, 0) and np.allclose(res.rux, 0)


def test_tiny_dense_generator_construction():
    """Ax0 - b = u >= 0.1 (x0 strictly feasible) and lambda_min(H) >= 1e-3."""
    spec = W.tiny_dense(0)
    prob = O.from_spec(spec)
    assert np.all(spec.A @ spec.extra["x0"] - spec.lA >= 0.1 - 1e-9)
    assert np.linalg.eigvalsh(prob.Hdense()).min() >= 1e-3 - 1e-9


# --------------------------------------------------------- Woodbury (P17)
def test_woodbury_direction_matches_dense():
    spec = W.svm_qp(5, 300, 8)
    prob = O.from_spec(spec)
    rng = np.random.default_rng(4)
    st = random_state(prob, rng, 0.5)
    st.lam_e = rng.standard_normal(1)
    d1, _, _ = O.newton_direction(prob, st, 0.01)
    d2 = O.woodbury_direction(prob, st, 0.01, h0=spec.h0, U=spec.U, wd=spec.wd)
    assert rel(d2.dx, d1.dx) < 1e-8
    assert rel(d2.dlam_lx, d1.dlam_lx) < 1e-8


# ---------------------------------------------------------- adjoint (P15/16)
def test_adjoint_unconstrained_closed_form():
    rng = np.random.default_rng(5)
    n = 6
    G = rng.standard_normal((n, n))
    H = G.T @ G + np.eye(n)
    prob = O.from_spec(W.QPSpec(n=n, c=rng.standard_normal(n), h_kind="dense", H=H))
    r = O.solve(prob)
    g = rng.standard_normal(n)
    out = O.adjoint_gradients(prob, r.state, r.mu, g)
    assert np.allclose(out["c"], -np.linalg.solve(H, g), rtol=1e-10)


def test_adjoint_matches_central_differences_on_centered_solves():
    """dL/d(c, l, u, b, w) from the adjoint agree with central differences of
    the exactly centered solution x*(theta) at fixed mu (h = 1e-6)."""
    rng = np.random.default_rng(6)
    base = W.rt_qp(4, 60, 8, 0.3, 8, maxdose=0.3)
    base.c = np.random.default_rng(4).standard_normal(base.n) * 0.5
    xref = rng.uniform(0, 1, base.n)
    prob = O.from_spec(base)
    r = O.solve(prob)
    mu = r.mu
    st = O.center(prob, r.state, mu)
    L = lambda x: float(np.sum((x - xref) ** 2))
    out = O.adjoint_gradients(prob, st, mu, 2 * (st.x - xref), P=base.P, w=base.w, d=base.d)
    # the case has active max-dose rows and active x >= 0 bounds
    assert (st.s_uA < 1e-4).sum() >= 2 and (st.s_lx < 1e-4).sum() >= 2
    assert np.linalg.norm(out["u"]) > 1e-2

    def solve_at(spec):
        p2 = O.from_spec(spec)
        return O.center(p2, st, mu).x

    import copy
    h = 1e-6
    for name, grad in (("c", out["c"]), ("uA", out["u"]), ("w", out["w"])):
        v = rng.standard_normal(grad.size)
        v /= np.linalg.norm(v)
        sp_, sm_ = copy.deepcopy(base), copy.deepcopy(base)
        setattr(sp_, name, getattr(base, name) + h * v)
        setattr(sm_, name, getattr(base, name) - h * v)
        fd = (L(solve_at(sp_)) - L(solve_at(sm_))) / (2 * h)
        assert abs(fd - grad @ v) <= 1e-4 * max(1e-3, abs(fd)), (name, fd, grad @ v)


def test_jacobi_spectrum_of_a_diagonal_system_is_one():
    """Box-only separable QP: K is diagonal, so diag(K)^-1 K = I."""
    n = 9
    spec = W.QPSpec(n=n, c=np.linspace(-1, 1, n), h_kind="dense", H=np.diag(np.linspace(1, 3, n)),
                    lx=-np.ones(n), ux=np.ones(n))
    prob = O.from_spec(spec)
    st = random_state(prob, np.random.default_rng(1), 0.5)
    lo, hi = O.jacobi_spectrum(prob, st, 0.3)
    assert lo == pytest.approx(1.0, abs=1e-14) and hi == pytest.approx(1.0, abs=1e-14)


def test_jacobi_spectrum_two_by_two_closed_form():
    """One variable, one lower-bounded row a x >= l: K = [[k11, a], [a, d]] with
    k11 = h + 2 a^2 / d and d = s / lam, so diag(K)^-1 K has eigenvalues
    1 -+ |a| / sqrt(k11 d), whatever h, a, s, lam are."""
    h, a = 2.5, 1.7
    spec = W.QPSpec(n=1, c=np.array([0.3]), h_kind="dense", H=np.array([[h]]),
                    A=np.array([[a]]), lA=np.array([-1.0]), uA=np.array([np.inf]))
    prob = O.from_spec(spec)
    st = random_state(prob, np.random.default_rng(2), 0.5)
    d = st.s_lA[0] / st.lam_lA[0]
    k11 = h + 2.0 * a * a / d
    off = abs(a) / np.sqrt(k11 * d)
    lo, hi = O.jacobi_spectrum(prob, st, 0.7)
    assert lo == pytest.approx(1.0 - off, rel=1e-13) and hi == pytest.approx(1.0 + off, rel=1e-13)
    c = O.condition_numbers(prob, st, 0.7)
    assert c["kappa_jacobi"] == pytest.approx((1.0 + off) / (1.0 - off), rel=1e-12)
    # K itself: eigenvalues (k11 + d)/2 -+ sqrt(((k11 - d)/2)^2 + a^2)
    mid, rad = 0.5 * (k11 + d), np.hypot(0.5 * (k11 - d), a)
    assert c["kappa"] == pytest.approx((mid + rad) / (mid - rad), rel=1e-11)


# ------------------------------------------- 1-norm condition estimate (Section 5.3)
def test_onenorm_estimate_is_exact_on_the_second_difference_matrix():
    """T = tridiag(-1, 2, -1) of odd order n: T^-1 has the entries
    min(i, j) (n + 1 - max(i, j)) / (n + 1) > 0, column j sums to
    j (n + 1 - j) / 2, so ||T^-1||_1 = (n + 1)^2 / 8 and ||T||_1 = 4.  With a
    positive inverse the first ascent step lands on the largest column."""
    n = 21
    T = 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    est = O.onenorm_inverse_estimate(lambda v: np.linalg.solve(T, v),
                                     lambda v: np.linalg.solve(T.T, v), n)
    assert est == pytest.approx((n + 1) ** 2 / 8.0, rel=1e-12)


def test_onenorm_estimate_is_a_lower_bound_within_a_small_factor():
    """Every value the estimator returns is ||A^-1 x||_1 / ||x||_1 for some x,
    so it never exceeds ||A^-1||_1 (computed here from the explicit inverse);
    on these seeded matrices it is within the factor 3 usually observed."""
    rng = np.random.default_rng(11)
    for t in range(60):
        n = int(rng.integers(2, 30))
        A = rng.standard_normal((n, n))
        if t % 2:
            A = A @ A.T + 0.05 * np.eye(n)
        Ai = np.linalg.inv(A)
        exact = np.abs(Ai).sum(axis=0).max()
        est = O.onenorm_inverse_estimate(lambda v: Ai @ v, lambda v: Ai.T @ v, n)
        assert exact / 3.5 <= est <= exact * (1 + 1e-12), (t, n, est, exact)
    d = rng.uniform(0.1, 5.0, 17)
    est = O.onenorm_inverse_estimate(lambda v: v / d, lambda v: v / d, 17)
    assert est == pytest.approx(1.0 / d.min(), rel=1e-14)


def test_condest_two_by_two_closed_form():
    """The 2 x 2 system of the spectrum pin: K = [[k11, a], [a, d]] has
    ||K||_1 = max(k11, d) + |a| and ||K^-1||_1 = (max(k11, d) + |a|) / det K;
    its symmetric Jacobi scaling [[1, o], [o, 1]], o = a / sqrt(k11 d), has
    1-norm condition (1 + |o|) / (1 - |o|)."""
    h, a = 2.5, -1.7
    spec = W.QPSpec(n=1, c=np.array([0.3]), h_kind="dense", H=np.array([[h]]),
                    A=np.array([[a]]), lA=np.array([-1.0]), uA=np.array([np.inf]))
    prob = O.from_spec(spec)
    st = random_state(prob, np.random.default_rng(2), 0.5)
    d = st.s_lA[0] / st.lam_lA[0]
    k11 = h + 2.0 * a * a / d
    o = abs(a) / np.sqrt(k11 * d)
    c = O.condest(prob, st, 0.7)
    assert c["kappa1"] == pytest.approx((max(k11, d) + abs(a)) ** 2 / (k11 * d - a * a), rel=1e-12)
    assert c["kappa1_jacobi"] == pytest.approx((1.0 + o) / (1.0 - o), rel=1e-12)


def test_condest_path_shows_jacobi_removing_the_barrier_ill_conditioning():
    """Section 5.3 on the quasi-Newton RT shape (n = 300, k = 12, 15 rows):
    along the interior point path the condition of K grows by many orders as
    mu falls, while the Jacobi preconditioned matrix stays orders of
    magnitude better.  Each estimate is checked against the exact 1-norm
    condition number computed from explicit inverses."""
    prob = O.from_spec(W.qn_rt(6, 300, 12, 15))
    res, rows = O.condest_path(prob)
    assert res.status == "converged" and len(rows) == res.iterations
    for r in rows:
        K = O.kkt_dense(prob, r["state"], r["mu"])
        s = 1.0 / np.sqrt(np.diag(K))
        for key, M in (("kappa1", K), ("kappa1_jacobi", s[:, None] * K * s[None, :])):
            exact = np.abs(M).sum(axis=0).max() * np.abs(np.linalg.inv(M)).sum(axis=0).max()
            assert exact / 3.5 <= r[key] <= exact * (1 + 1e-8), (r["it"], key, r[key], exact)
    k = np.array([r["kappa1"] for r in rows])
    kj = np.array([r["kappa1_jacobi"] for r in rows])
    assert rows[-1]["mu"] < 1e-6 and k[-1] >= 1e10 * k[0]
    assert np.all(kj <= k) and kj[-1] <= 1e-4 * k[-1]


# ------------------------------------------------ PCG stop rule (Section 5.1)
def _true_relres(K, rhs, x):
    """||rhs - K x||_2 / ||rhs||_2 computed here, not taken from the solver."""
    return float(np.linalg.norm(rhs - K @ x) / np.linalg.norm(rhs))


def test_pcg_stops_at_first_iterate_below_tol_on_the_unpreconditioned_residual():
    """Section 5.1: the PCG stops on the unpreconditioned residual (relative
    to ||rhs||_2, the reading of the tolerance).  The iterates x_j are taken
    from runs capped at j iterations, and their residuals are recomputed here
    from K: the returned count k must be the first j whose true residual is
    at or below tol.  The system is scaled so that a stop on ||z|| = ||D^-1 r||
    or on the D^-1-norm of r would stop at a different iteration (asserted),
    so either mistake fails this pin."""
    rng = np.random.default_rng(20)
    prob = general(24, n=30, m=25, me=2, mg=10)
    st = random_state(prob, rng, 1.5)        # a wide spread of D entries
    mu = 0.05
    K = O.spectrum.kkt_dense(prob, st, mu)
    rhs, _ = O.newton_rhs_doubly(prob, st, mu)
    dg = np.diag(K)
    tol = 1e-7
    x, k, conv, rr = pcg(lambda v: K @ v, rhs, dg, tol, 5000)
    assert conv and 2 < k < 5000
    iters = [pcg(lambda v: K @ v, rhs, dg, tol, j)[0] for j in range(k + 1)]
    assert np.array_equal(iters[k], x)
    true = [_true_relres(K, rhs, xj) for xj in iters]
    first = next(j for j, t in enumerate(true) if t <= tol)
    assert first == k, (first, k)
    assert rr == pytest.approx(true[k], rel=1e-6)
    # a solve capped one iteration early returns that iterate, unconverged
    xm, km, cm, rm = pcg(lambda v: K @ v, rhs, dg, tol, k - 1)
    assert km == k - 1 and not cm and np.array_equal(xm, iters[k - 1])
    assert rm == pytest.approx(true[k - 1], rel=1e-6) and rm > tol
    # the pin discriminates: preconditioned-norm stop rules cross elsewhere
    zrel = [np.linalg.norm((rhs - K @ xj) / dg) / np.linalg.norm(rhs / dg) for xj in iters]
    drel = [np.sqrt(((rhs - K @ xj) ** 2 / dg).sum() / (rhs ** 2 / dg).sum()) for xj in iters]
    assert next((j for j, t in enumerate(zrel) if t <= tol), None) != k
    assert next((j for j, t in enumerate(drel) if t <= tol), None) != k


def test_pcg_starts_at_zero_and_first_step_is_the_jacobi_steepest_descent_step():
    """x0 = 0 (reading of Section 5.1); with z0 = D^-1 rhs the first iterate is
    x1 = (rhs^T z0 / z0^T K z0) z0 in closed form, which fixes both the start
    and the Jacobi preconditioner D = diag(K) of Section 3.1."""
    rng = np.random.default_rng(14)
    prob = general(18, n=12, m=9, me=1, mg=5)
    st = random_state(prob, rng, 1.0)
    K = O.spectrum.kkt_dense(prob, st, 0.3)
    rhs, _ = O.newton_rhs_doubly(prob, st, 0.3)
    dg = np.diag(K)
    x0, k0, c0, r0 = pcg(lambda v: K @ v, rhs, dg, 1e-7, 0)
    assert k0 == 0 and not c0 and np.all(x0 == 0) and r0 == pytest.approx(1.0, rel=1e-15)
    z0 = rhs / dg
    x1 = (rhs @ z0) / (z0 @ K @ z0) * z0
    xp, k1, _, _ = pcg(lambda v: K @ v, rhs, dg, 1e-7, 1)
    assert k1 == 1 and np.allclose(xp, x1, rtol=1e-13, atol=0)


# -------------------------------------- adjoint: lower rows and equality rows
def test_adjoint_equality_only_closed_form():
    """Only C x = b: at fixed mu the penalty-barrier conditions are linear,
    (H + C^T C / mu) x = -p + C^T b / mu, so for L(x) with gradient g,
    dL/dp = -M^-1 g and dL/db = C M^-1 g / mu with M = H + C^T C / mu."""
    rng = np.random.default_rng(15)
    n, me = 7, 3
    G = rng.standard_normal((n, n))
    H = G.T @ G + np.eye(n)
    C = rng.standard_normal((me, n))
    prob = O.from_spec(W.QPSpec(n=n, c=rng.standard_normal(n), h_kind="dense", H=H, C=C,
                                b=rng.standard_normal(me)))
    r = O.solve(prob)
    g = rng.standard_normal(n)
    out = O.adjoint_gradients(prob, r.state, r.mu, g)
    M = H + C.T @ C / r.mu
    v = np.linalg.solve(M, g)
    # both solves are backward stable: they agree to about cond(M) * eps
    bound = 100 * np.linalg.cond(M) * np.finfo(float).eps
    assert rel(out["c"], -v) <= bound
    assert rel(out["b"], C @ v / r.mu) <= bound


def test_adjoint_lower_rows_and_equality_rhs_match_central_differences():
    """dL/dl_A (rows with a finite lower side, several of them active) and
    dL/db (equality rows) from the adjoint agree with central differences of
    the exactly centered solution at fixed mu (h = 1e-6), along seeded random
    directions and single coordinates.  The closed form above pins dL/db only
    without inequalities; this pins the sign and scale with them."""
    import copy
    rng = np.random.default_rng(16)
    base = W.random_bounded_qp(1, 8, 7, 2, 4)
    prob = O.from_spec(base)
    S = O.index_sets(prob)
    r = O.solve(prob)
    mu = r.mu
    st = O.center(prob, r.state, mu)
    assert (st.s_lA < 1e-4).sum() >= 2 and prob.me == 2
    xref = rng.uniform(-1, 1, base.n)
    L = lambda x: float(np.sum((x - xref) ** 2))
    out = O.adjoint_gradients(prob, st, mu, 2 * (st.x - xref))
    assert np.linalg.norm(out["l"]) > 1e-2 and np.linalg.norm(out["b"]) > 1e-2
    assert np.all(out["l"][~np.isfinite(prob.l)] == 0)

    def solve_at(spec):
        return O.center(O.from_spec(spec), st, mu).x

    h = 1e-6
    for name, key, mask in (("lA", "l", np.isfinite(base.lA)), ("b", "b", np.ones(base.me, bool))):
        grad = out[key]
        dirs = []
        for _ in range(3):
            v = rng.standard_normal(grad.size) * mask
            dirs.append(v / np.linalg.norm(v))
        for i in np.flatnonzero(mask)[:4]:
            e = np.zeros(grad.size)
            e[i] = 1.0
            dirs.append(e)
        for v in dirs:
            sp_, sm_ = copy.deepcopy(base), copy.deepcopy(base)
            setattr(sp_, name, getattr(base, name) + h * v)
            setattr(sm_, name, getattr(base, name) - h * v)
            fd = (L(solve_at(sp_)) - L(solve_at(sm_))) / (2 * h)
            assert abs(fd - grad @ v) <= 1e-4 * max(1e-3, abs(fd)), (name, fd, grad @ v)
