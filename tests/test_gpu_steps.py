"""GPU parity of every step of the hot path against the CPU oracle, through
the C ABI (steps a1-a8 at arbitrary interior states, then Algorithm 1).
Vectors are compared block by block (each block of the residual stack, the
doubly augmented vector and the iterate against its own norm), so an error
confined to a small block is not hidden by a large one."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2308_00637_amd import workloads as W
from tests.helpers import (block_rel, dir_to_masked, from_masked, kkt_blocks, kkt_from_masked,
                           kkt_to_masked, lam_blocks, random_state, rel, res_blocks,
                           res_to_masked, s_blocks, to_masked)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cases():
    return {
        "general_dense": lambda: W.random_bounded_qp(1, 37, 29, 2, 11),
        "general_csr_lowrank": lambda: W.random_bounded_qp(2, 53, 41, 1, 9, a_sparse=True,
                                                           h_kind="lowrank"),
        "rt_ptwp": lambda: W.rt_qp(5, 700, 61, 0.08, 23, maxdose=0.6),
        "svm_lowrank_eq": lambda: W.svm_qp(6, 333, 7),
        "tiny_dense": lambda: W.tiny_dense(0),
        "no_rows_bounds_only": lambda: W.QPSpec(n=70, c=np.linspace(-3, 3, 70), h_kind="dense",
                                                H=np.diag(np.linspace(0.5, 2, 70)),
                                                lx=-np.ones(70), ux=np.ones(70)),
        # empty and several-hundred-entry rows, variables in no row, free rows
        "ragged_ptwp": lambda: W.ragged_qp(9),
        "single_variable": lambda: W.QPSpec(
            n=1, c=np.array([-1.0]), h_kind="ptwp",
            P=sp.csr_matrix(np.array([[1.0], [0.5], [2.0]])), w=np.ones(3), d=np.array([0.3, 0.1, 0.9]),
            A=sp.csr_matrix(np.array([[2.0]])), lA=np.array([-np.inf]), uA=np.array([1.0]),
            lx=np.zeros(1), ux=np.full(1, np.inf)),
        "max_equalities": lambda: W.random_bounded_qp(3, 150, 40, 64, 20),
        # H = diag(h0) + U diag(w) U^T with mixed-sign w (limited-memory BFGS form)
        "quasi_newton_mixed_w": lambda: W.qn_rt(6, 300, 12, 15),
        # SVM dual with a dense RBF-kernel Hessian, one equality row, a box
        "svm_rbf_dense": lambda: W.svm_rbf(7, 300),
    }


CASES = _cases()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", params=list(CASES))
def setup(request):
    from paper_2308_00637_amd.qpk import QP
    spec = CASES[request.param]()
    prob = O.from_spec(spec)
    qp = QP(spec)
    rng = np.random.default_rng(42)
    st = random_state(prob, rng, 0.5)
    mu = 0.37
    x, lam, s = to_masked(prob, st)
    qp.set_state(dev(x), dev(lam), dev(s), mu)
    print(f"case={request.param} n={prob.n} m={prob.m} me={prob.me}", flush=True)
    return request.param, spec, prob, qp, st, mu


def test_a1_residuals(setup):
    name, spec, prob, qp, st, mu = setup
    r, norms = qp.residuals()
    res = O.residuals(prob, st, mu)
    ref = res_to_masked(prob, res)
    assert block_rel(host(r), ref, res_blocks(prob)) <= 1e-12
    pr, du, co = O.infeasibilities(res)
    assert norms[0] == pytest.approx(O.stacked_norm(res), rel=1e-12)
    assert norms[1:] == pytest.approx([pr, du, co], rel=1e-12, abs=1e-300)


def test_a2_a3_rhs_and_jacobi(setup):
    name, spec, prob, qp, st, mu = setup
    rhs, dg = qp.newton_rhs()
    ref_rhs, _ = O.newton_rhs_doubly(prob, st, mu)
    ref_dg = O.jacobi_diagonal(prob, st, mu)
    kb = kkt_blocks(prob)
    assert block_rel(kkt_from_masked(prob, host(rhs)), ref_rhs, kb) <= 1e-12
    assert block_rel(kkt_from_masked(prob, host(dg)), ref_dg, kb) <= 1e-12


def test_a4_matvec(setup):
    name, spec, prob, qp, st, mu = setup
    rng = np.random.default_rng(7)
    N = prob.n + prob.me + O.index_sets(prob).L.size + O.index_sets(prob).U.size
    for _ in range(3):
        v = rng.standard_normal(N)
        y = qp.kkt_matvec(dev(kkt_to_masked(prob, v)))
        ref = O.kkt_matvec(prob, st, mu, v)
        yh = host(y)
        assert block_rel(kkt_from_masked(prob, yh), ref, kkt_blocks(prob)) <= 1e-12
        # rows of absent sides are identity rows on a zero input
        assert np.all(yh[np.abs(kkt_to_masked(prob, np.ones(N))) == 0] == 0)


def test_a5_pcg_matches_cholesky_and_oracle_pcg(setup):
    from oracle.pcg import pcg
    from paper_2308_00637_amd.qpk import default_pcg_options
    name, spec, prob, qp, st, mu = setup
    rhs, _ = qp.newton_rhs()
    ref_rhs, res = O.newton_rhs_doubly(prob, st, mu)
    Q, B, D, r1, r2, _ = O.reduced_system(prob, st, res, mu)
    K, _ = O.doubly_augmented(Q, B, D, r1, r2)
    xd = np.linalg.solve(K, ref_rhs)
    sol, info = qp.kkt_pcg_solve(rhs, default_pcg_options(tol=1e-12, maxit=20000))
    assert info.converged == 1 and info.rel_residual <= 1e-11
    assert block_rel(kkt_from_masked(prob, host(sol)), xd, kkt_blocks(prob)) <= 1e-7
    # iteration count at the paper's tolerance agrees with a textbook PCG
    sol, info = qp.kkt_pcg_solve(rhs, default_pcg_options(tol=1e-7))
    _, it, conv, _ = pcg(lambda v: K @ v, ref_rhs, np.diag(K), 1e-7, 5000)
    assert conv and info.converged == 1
    assert abs(info.iterations - it) <= max(2, it // 50), (info.iterations, it)


def test_a6_direction(setup):
    from paper_2308_00637_amd.qpk import default_pcg_options
    name, spec, prob, qp, st, mu = setup
    dx, dl, ds, info = qp.newton_direction(default_pcg_options(tol=1e-13, maxit=20000))
    d, _, _ = O.newton_direction(prob, st, mu)
    rx, rl, rs = dir_to_masked(prob, d)
    assert rel(host(dx), rx) <= 1e-7
    assert block_rel(host(dl), rl, lam_blocks(prob)) <= 1e-7
    assert block_rel(host(ds), rs, s_blocks(prob)) <= 1e-7


def test_a7_a8_step_lengths_and_update(setup):
    name, spec, prob, qp, st, mu = setup
    d, _, _ = O.newton_direction(prob, st, mu)
    rx, rl, rs = dir_to_masked(prob, d)
    ax, al = qp.step_lengths(dev(rl), dev(rs), 0.99)
    oax, oal = O.step_lengths(st, d, 0.99)
    assert ax == pytest.approx(oax, rel=1e-14) and al == pytest.approx(oal, rel=1e-14)
    x0, l0, s0, _ = qp.get_state()
    qp.take_step(dev(rx), dev(rl), dev(rs), ax, al)
    x1, l1, s1, _ = qp.get_state()
    st1 = O.take_step(st, d, oax, oal)
    ex, el, es = to_masked(prob, st1)
    assert rel(host(x1), ex) <= 1e-14
    assert block_rel(host(l1), el, lam_blocks(prob)) <= 1e-14
    assert block_rel(host(s1), es, s_blocks(prob)) <= 1e-14
    # restore the module-scoped state
    qp.set_state(x0, l0, s0, mu)


def test_a9_ipm_solve_matches_oracle(setup):
    name, spec, prob, qp, st, mu = setup
    ref = O.solve(prob)
    out = qp.solve(log=True)
    info = out["info"]
    assert info.result == 0 and ref.status == "converged"
    assert abs(info.objective - ref.objective) <= 1e-6 * max(1.0, abs(ref.objective))
    print(f"ipm iters gpu={info.iterations} oracle={ref.iterations} cg={info.total_cg_iters} "
          f"cg_cap_hits={info.cg_maxiter_hits} obj={info.objective:.12g}/{ref.objective:.12g}")
    # KKT residual of the returned point, evaluated by the oracle's own function
    gst = from_masked(prob, host(out["x"]), host(out["lam"]), host(out["s"]))
    kkt = O.stacked_norm(O.residuals(prob, gst, info.mu_final))
    assert kkt <= 1e-6, kkt
    assert kkt == pytest.approx(info.rnorm, rel=1e-9)
    assert info.mu_final < 1e-6 and info.mu_final >= 1e-8
    mus = out["log"]["mu"]
    assert mus[0] == 1.0 and np.all(np.diff(mus) <= 0)
    assert set(np.round(np.log10(mus)).astype(int)) == set(range(0, -8, -1))


# IPM iterations before the first Newton system at which the oracle's own
# Jacobi PCG (tolerance 1e-7, 5000 iterations) stops at its cap.  A capped PCG
# returns an iterate that depends on rounding order (5000 steps of a recurrence
# that has lost orthogonality), so schedules are compared up to there.
SCHEDULE_PREFIX = {"tiny_dense": 24, "ragged_ptwp": 17, "max_equalities": 16}


def oracle_pcg_direction(record):
    """Newton directions by the oracle's textbook Jacobi PCG on eq. (9)
    (Section 3.1; tolerance and cap of Section 5.1), recording iterations."""
    from oracle.pcg import pcg

    def direction(prob, st, mu, res):
        rhs, _ = O.newton_rhs_doubly(prob, st, mu)
        dg = O.jacobi_diagonal(prob, st, mu)
        sol, k, conv, _ = pcg(lambda v: O.kkt_matvec(prob, st, mu, v), rhs, dg, tol=1e-7, maxit=5000)
        record.append((k, conv))
        return O.direction_from_solution(prob, st, res, sol)
    return direction


def test_a9_schedule_matches_oracle_pcg_driven_ipm(setup):
    """Algorithm 1 with PCG directions on both sides: the GPU solve and the
    oracle's IPM driven by its own Jacobi PCG take the same steps, drop mu at
    the same iterations (strict ||r|| < mu, mu / 10) and end at the same
    point.  Each Newton step is a PCG solve to a relative residual of 1e-7 and
    CG iterates are sensitive to rounding order, so the two runs take slightly
    different inexact steps: a system's stop moves by a few iterations and
    the residual norms after a step agree to a few digits.  A decrease of mu
    is a threshold test, so the two runs may part where ||r|| is within a few
    percent of mu (a near tie), or late in the solve, once ||r|| is so small
    that the steps' PCG error decides it (the two runs' ||r|| then differ by
    a factor, not in the last digits).  The test walks both logs to the first
    parting, requires it to be one of the two, and requires the runs to end
    within two iterations of each other at the same point."""
    from paper_2308_00637_amd.qpk import default_ipm_options
    name, spec, prob, qp, st, mu = setup
    its = SCHEDULE_PREFIX.get(name, 200)
    record = []
    ref = O.solve(prob, O.IPMOptions(max_iter=its), direction=oracle_pcg_direction(record))
    assert all(conv for _, conv in record)
    out = qp.solve(default_ipm_options(max_iter=its), log=True)
    info, lg = out["info"], out["log"]
    assert (info.result == 0) == (ref.status == "converged")
    assert info.cg_maxiter_hits == 0
    omus = [e["mu"] for e in ref.log]
    part = next((k for k, (a, b) in enumerate(zip(lg["mu"], omus)) if a != b),
                min(len(omus), len(lg["mu"])))
    same = part      # iterations solved with the same mu
    cg_gap = [abs(int(a) - k) for a, (k, _) in zip(lg["cg_iters"][:same], record)]
    big = [(a, e["rnorm"]) for a, e in zip(lg["rnorm"][:same], ref.log) if e["rnorm"] >= 1e-4]
    r_gap = max([abs(a - b) / b for a, b in big] or [0.0])
    x = host(out["x"])
    dxm = float(np.max(np.abs(x - ref.state.x) / np.maximum(1.0, np.abs(ref.state.x))))
    msg = (f"{name}: ipm gpu={info.iterations} oracle={ref.iterations}; same mu for {same} iterations; "
           f"CG counts within {max(cg_gap)}; ||r|| >= 1e-4 within {r_gap:.1e} rel; max|dx| {dxm:.1e}")
    if part < min(len(omus), len(lg["mu"])):
        k = part - 1    # the iteration whose test ||r|| < mu the runs decided differently
        tie_o, tie_g = ref.log[k]["rnorm"] / omus[k], lg["rnorm"][k] / lg["mu"][k]
        msg += f"; parted after iteration {k + 1}: ||r||/mu oracle {tie_o:.4f} gpu {tie_g:.4f}"
        late = ref.log[k]["rnorm"] <= 1e-4 * ref.log[0]["rnorm"]
        assert (abs(tie_o - 1.0) <= 0.05 and abs(tie_g - 1.0) <= 0.05) or late, msg
    print(msg, flush=True)
    assert abs(info.iterations - ref.iterations) <= 2
    # ill-conditioned late systems (thousands of CG iterations) stop a few
    # percent apart and their steps' residuals agree to a few percent
    assert all(g <= max(3, k // 10) for g, (k, _) in zip(cg_gap, record))
    assert r_gap <= 0.25
    assert dxm <= 1e-6


def test_unconstrained_qp_takes_exactly_eight_iterations():
    """No rows, no bounds: the first Newton step solves H x = -p (to the PCG
    tolerance), every later residual is below mu, so mu falls 1 -> 1e-7 by
    tenths and the solve returns after exactly 8 iterations (the strict test
    mu < 1e-6 fails at mu = 1.0000000000000002e-06), at x = -H^-1 p."""
    from paper_2308_00637_amd.qpk import QP
    rng = np.random.default_rng(8)
    n = 60
    G = rng.standard_normal((40, n))
    H = G.T @ G + np.eye(n)
    c = rng.standard_normal(n)
    out = QP(W.QPSpec(n=n, c=c, h_kind="dense", H=H, name="unconstrained")).solve(log=True)
    info = out["info"]
    assert info.result == 0 and info.iterations == 8
    mus = [1.0]
    for _ in range(7):
        mus.append(mus[-1] / 10.0)
    assert list(out["log"]["mu"]) == mus
    x_star = np.linalg.solve(H, -c)
    assert rel(host(out["x"]), x_star) <= 1e-10


def test_box_only_separable_qp_reaches_the_clipped_minimiser():
    """Diagonal H with bounds only: x* = clip(-c/h, lx, ux) coordinate-wise.
    Coordinate j of the barrier point sits about mu / (h_j dist_j) from x*_j
    when x*_j is inside the box (dist_j: distance to the nearer bound) and
    about mu / lam_j when it is at a bound with multiplier
    lam_j = |h_j x*_j + c_j|; the returned point is checked against ten times
    that, and against the oracle's own solve elementwise."""
    from paper_2308_00637_amd.qpk import QP
    spec = CASES["no_rows_bounds_only"]()
    h = np.diag(spec.H)
    x_star = np.clip(-spec.c / h, spec.lx, spec.ux)
    out = QP(spec).solve()
    info = out["info"]
    assert info.result == 0
    x = host(out["x"])
    scale = np.maximum(h * np.minimum(x_star - spec.lx, spec.ux - x_star), np.abs(h * x_star + spec.c))
    with np.errstate(divide="ignore"):   # a zero multiplier at a bound: no bound there
        assert np.all(np.abs(x - x_star) <= 10 * info.mu_final / scale)
    ref = O.solve(O.from_spec(spec))
    assert np.max(np.abs(x - ref.state.x)) <= 1e-6
