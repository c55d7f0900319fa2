"""Condition number diagnostic (Section 5.3): the extreme eigenvalues of the
doubly augmented matrix, with the Jacobi preconditioner and without it
(pcg_options.no_precond), estimated on the GPU from the CG coefficients
(Ritz values of the Lanczos matrix CG builds implicitly), against the
oracle's dense eigenvalues at the same state.  Ritz values lie inside the
spectrum and approach its ends as CG converges."""
import numpy as np
import pytest

import oracle as O
from paper_2308_00637_amd import workloads as W
from tests.helpers import kkt_from_masked, random_state, to_masked

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "general_dense": lambda: W.random_bounded_qp(1, 37, 29, 2, 11),
    "rt_ptwp": lambda: W.rt_qp(5, 700, 61, 0.08, 23, maxdose=0.6),
    "quasi_newton_mixed_w": lambda: W.qn_rt(6, 300, 12, 15),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("case", list(CASES))
def test_ritz_values_bracket_inside_the_dense_spectrum(case):
    from paper_2308_00637_amd.qpk import QP, default_pcg_options
    spec = CASES[case]()
    prob = O.from_spec(spec)
    qp = QP(spec)
    st = random_state(prob, np.random.default_rng(42), 0.5)
    mu = 0.37
    x, lam, s = to_masked(prob, st)
    qp.set_state(dev(x), dev(lam), dev(s), mu)
    rhs, _ = qp.newton_rhs()
    _, info = qp.kkt_pcg_solve(rhs, default_pcg_options(tol=1e-10, spectrum=1))
    lo, hi = O.jacobi_spectrum(prob, st, mu)
    print(f"{case}: its={info.iterations} ritz=[{info.lambda_min:.6g}, {info.lambda_max:.6g}] "
          f"dense=[{lo:.6g}, {hi:.6g}]", flush=True)
    assert info.converged == 1
    assert lo * (1 - 1e-9) <= info.lambda_min <= info.lambda_max <= hi * (1 + 1e-9)
    # converged to 1e-10: the extreme Ritz values have found the spectrum's ends
    assert info.lambda_max >= 0.99 * hi
    assert info.lambda_min <= 1.1 * lo


def test_ipm_logs_kappa_per_newton_system():
    from paper_2308_00637_amd.qpk import QP, default_ipm_options
    spec = CASES["rt_ptwp"]()
    prob = O.from_spec(spec)
    opts = default_ipm_options()
    opts.pcg.spectrum = 1
    out = QP(spec).solve(opts, log=True)
    kap = out["log"]["kappa"]
    print("kappa per IPM iteration:", np.array2string(kap, precision=3), flush=True)
    assert out["info"].result == 0
    assert np.all(np.isfinite(kap)) and np.all(kap >= 1.0)
    # the first Newton system is at the default start point with mu = 1
    lo, hi = O.jacobi_spectrum(prob, O.initial_point(prob), 1.0)
    assert kap[0] <= hi / lo * (1 + 1e-9) and kap[0] >= 0.5 * hi / lo


@pytest.mark.parametrize("case", list(CASES))
def test_plain_cg_ritz_values_and_solution_against_dense_k(case):
    from paper_2308_00637_amd.qpk import QP, default_pcg_options
    spec = CASES[case]()
    prob = O.from_spec(spec)
    qp = QP(spec)
    st = random_state(prob, np.random.default_rng(42), 0.5)
    mu = 0.37
    x, lam, s = to_masked(prob, st)
    qp.set_state(dev(x), dev(lam), dev(s), mu)
    rhs, _ = qp.newton_rhs()
    sol, info = qp.kkt_pcg_solve(rhs, default_pcg_options(tol=1e-10, spectrum=1, no_precond=1))
    _, jinfo = qp.kkt_pcg_solve(rhs, default_pcg_options(tol=1e-10))
    K = O.kkt_dense(prob, st, mu)
    ev = np.linalg.eigvalsh(K)
    kap = O.condition_numbers(prob, st, mu)
    print(f"{case}: plain its={info.iterations} (Jacobi {jinfo.iterations}) "
          f"ritz=[{info.lambda_min:.6g}, {info.lambda_max:.6g}] dense=[{ev[0]:.6g}, {ev[-1]:.6g}] "
          f"kappa={kap['kappa']:.3g} kappa_jacobi={kap['kappa_jacobi']:.3g}", flush=True)
    assert info.converged == 1
    assert ev[0] * (1 - 1e-9) <= info.lambda_min <= info.lambda_max <= ev[-1] * (1 + 1e-9)
    assert info.lambda_max >= 0.99 * ev[-1]
    assert info.lambda_min <= 1.1 * ev[0]
    # plain CG reaches the same solution (the host copy is in the masked layout)
    ref = np.linalg.solve(K, O.newton_rhs_doubly(prob, st, mu)[0])
    got = kkt_from_masked(prob, sol.cpu().numpy())
    assert np.linalg.norm(got - ref) <= 1e-10 * kap["kappa"] * np.linalg.norm(ref)


def test_ipm_logs_kappa_of_k_itself_by_plain_cg():
    from paper_2308_00637_amd.qpk import QP, default_ipm_options
    spec = CASES["rt_ptwp"]()
    prob = O.from_spec(spec)
    opts = default_ipm_options()
    opts.pcg.spectrum = 1
    out = QP(spec).solve(opts, log=True, log_kappa_plain=True)
    ref = QP(spec).solve(default_ipm_options())
    kj, kp = out["log"]["kappa"], out["log"]["kappa_plain"]
    print("kappa (Jacobi):", np.array2string(kj, precision=3), flush=True)
    print("kappa (plain): ", np.array2string(kp, precision=3), flush=True)
    # the extra solves leave the method's own path alone
    assert out["info"].result == 0 and out["info"].iterations == ref["info"].iterations
    assert out["info"].objective == pytest.approx(ref["info"].objective, rel=1e-10)
    assert np.all(np.isfinite(kp)) and np.all(kp >= 1.0)
    # first Newton system: default start point, mu = 1; Ritz estimates from inside the spectrum
    c = O.condition_numbers(prob, O.initial_point(prob), 1.0)
    assert 0.5 * c["kappa"] <= kp[0] <= c["kappa"] * (1 + 1e-9)
    assert 0.5 * c["kappa_jacobi"] <= kj[0] <= c["kappa_jacobi"] * (1 + 1e-9)


PATH_CASES = {
    "rt_small": W.rt_small,
    "quasi_newton_n300": lambda: W.qn_rt(6, 300, 12, 15),
}


@pytest.mark.timeout(600)
@pytest.mark.parametrize("case", list(PATH_CASES))
def test_condest_path_against_gpu_ritz_estimates(case):
    """Section 5.3 per Newton system along the interior point path: the
    oracle's 1-norm condition estimates (Hager/Higham with Cholesky) of K and
    of its Jacobi scaling, the exact 2-norm condition numbers, and the GPU's
    Ritz estimates from CG on the same system with the solver's settings
    (tol 1e-7, at most 5000 iterations), with and without the preconditioner.
    Ritz values lie inside the spectrum, so the GPU figures never exceed the
    exact 2-norm condition (up to the rounding of the CG coefficients, about
    1e-12 of the largest eigenvalue for the smallest); for a symmetric matrix
    that is at most the exact 1-norm condition.  With the preconditioner the
    Ritz estimate finds the spectrum's ends on every system of the path.
    Without it the estimate of K's own condition falls short late in the path
    by orders of magnitude, both where plain CG stops at the cap and where it
    meets the tolerance in a few hundred iterations because the right-hand
    side barely excites the extreme eigenvectors: the 1-norm estimate is the
    one that measures K itself there."""
    from paper_2308_00637_amd.qpk import QP, default_pcg_options
    spec = PATH_CASES[case]()
    prob = O.from_spec(spec)
    res, rows = O.condest_path(prob)
    assert res.status == "converged"
    qp = QP(spec)
    table = []
    for r in rows:
        st, mu = r["state"], r["mu"]
        K = O.kkt_dense(prob, st, mu)
        sc = 1.0 / np.sqrt(np.diag(K))
        ev = np.linalg.eigvalsh(K)
        evj = np.linalg.eigvalsh(sc[:, None] * K * sc[None, :])
        x, lam, s = to_masked(prob, st)
        qp.set_state(dev(x), dev(lam), dev(s), mu)
        rhs, _ = qp.newton_rhs()
        _, ij = qp.kkt_pcg_solve(rhs, default_pcg_options(spectrum=1))
        _, ip = qp.kkt_pcg_solve(rhs, default_pcg_options(spectrum=1, no_precond=1))
        for info, e in ((ij, evj), (ip, ev)):
            assert e[0] - 1e-12 * e[-1] <= info.lambda_min <= info.lambda_max <= e[-1] * (1 + 1e-9)
        table.append((r["it"], mu, r["kappa1"], ev[-1] / ev[0], ip.lambda_max / ip.lambda_min,
                      ip.iterations, r["kappa1_jacobi"], evj[-1] / evj[0],
                      ij.lambda_max / ij.lambda_min, ij.iterations, ip.converged, ij.converged))
    print(f"\n{case}: it mu | K: condest1 exact2 ritz(cg its) | Jacobi: condest1 exact2 ritz(pcg its)")
    for t in table:
        print("  %2d %.0e | %.3e %.3e %.3e (%4d) | %.3e %.3e %.3e (%4d)" % t[:10], flush=True)
    t = np.array(table)
    # the preconditioned matrix stays near 1e8 or below, and its Ritz estimate
    # reaches the exact 2-norm condition to within a factor 2 on every system
    assert np.all(t[:, 8] >= 0.5 * t[:, 7])
    # Jacobi removes the barrier's ill-conditioning: at the last Newton system
    # both the oracle's estimate and the GPU's are orders below K's own
    assert t[-1, 6] <= 1e-4 * t[-1, 2] and t[-1, 8] <= 1e-4 * t[-1, 2]
