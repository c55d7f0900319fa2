"""Run-time failure paths of the boundary, each beside the oracle's outcome on
the same problem:

* a nonconvex H (K indefinite at the first Newton system): ipm_solve and
  kkt_pcg_solve return QP_ERR_NOT_SPD (PCG met p^T K p <= 0, Section 3.1:
  PCG needs K positive definite), the oracle's Cholesky of eq. (9) fails;
  the kernels exit through the status flag, so the handle stays usable;
* a PCG capped at one iteration (Section 5.1's cap, Algorithm 1 goes on with
  the iterate): every Newton system counts as a cap hit, and the iterates
  follow the oracle's IPM driven by its own one-iteration PCG;
* rows with an empty feasible set: the barrier parameter never drops and the
  solve stops at the IPM iteration cap (QP_IPM_MAX_ITER), as the oracle does.

The oracle halves run on the CPU without a GPU."""
import warnings

import numpy as np
import pytest

import oracle as O
from oracle.pcg import pcg
from paper_2308_00637_amd import workloads as W
from tests.helpers import rel


def nonconvex_case():
    """min 1/2 x^T H x + c^T x with H = blockdiag([[1, 2], [2, 1]]) (eigenvalues
    3 and -1), no constraints; c alternates in sign so the first PCG search
    direction is an eigenvector of eigenvalue -1."""
    n = 12
    H = np.kron(np.eye(n // 2), np.array([[1.0, 2.0], [2.0, 1.0]]))
    c = np.tile([1.0, -1.0], n // 2)
    return W.QPSpec(n=n, c=c, h_kind="dense", H=H, name="nonconvex")


def infeasible_case():
    """x_0 >= 1 and x_0 <= 0 as two rows of A; H = I."""
    n = 6
    A = np.zeros((2, n))
    A[:, 0] = 1.0
    c = np.random.default_rng(0).standard_normal(n)
    return W.QPSpec(n=n, c=c, h_kind="dense", H=np.eye(n), A=A,
                    lA=np.array([1.0, -np.inf]), uA=np.array([np.inf, 0.0]), name="infeasible")


def capped_case():
    return W.random_bounded_qp(41, 30, 25, 2, 10)


def oracle_pcg_direction(maxit):
    def direction(prob, st, mu, res):
        rhs, _ = O.newton_rhs_doubly(prob, st, mu)
        dg = O.jacobi_diagonal(prob, st, mu)
        sol, _, _, _ = pcg(lambda v: O.kkt_matvec(prob, st, mu, v), rhs, dg, tol=1e-7, maxit=maxit)
        return O.direction_from_solution(prob, st, res, sol)
    return direction


# ---- oracle side (CPU) ----

def test_oracle_nonconvex_raises_not_spd():
    prob = O.from_spec(nonconvex_case())
    assert np.linalg.eigvalsh(prob.Hdense()).min() < 0
    with pytest.raises(O.NotSPDError):
        O.solve(prob)


def test_oracle_infeasible_stops_at_the_cap_with_mu_unchanged():
    prob = O.from_spec(infeasible_case())
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        r = O.solve(prob, O.IPMOptions(max_iter=8))
    assert r.status == "max_iter" and r.iterations == 8
    assert all(e["mu"] == 1.0 for e in r.log) and all(e["rnorm"] >= 1.0 for e in r.log)


# ---- GPU ----

def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.gpu
def test_nonconvex_is_not_spd_and_the_handle_survives():
    from paper_2308_00637_amd.qpk import QP, QPError, QP_ERR_NOT_SPD
    spec = nonconvex_case()
    qp = QP(spec)
    with pytest.raises(QPError) as e:
        qp.solve()
    assert e.value.status == QP_ERR_NOT_SPD
    qp.init_state(1.0)
    rhs, _ = qp.newton_rhs()
    with pytest.raises(QPError) as e:
        qp.kkt_pcg_solve(rhs)
    assert e.value.status == QP_ERR_NOT_SPD
    # the kernels stopped through the status flag: later calls still run
    r, norms = qp.residuals()
    prob = O.from_spec(spec)
    res = O.residuals(prob, O.initial_point(prob), 1.0)
    assert abs(norms[0] - O.stacked_norm(res)) <= 1e-12 * O.stacked_norm(res)


@pytest.mark.gpu
def test_pcg_capped_at_one_iteration_counts_every_newton_system():
    from paper_2308_00637_amd.qpk import QP, default_ipm_options, default_pcg_options
    spec = capped_case()
    prob = O.from_spec(spec)
    its = 6
    opts = default_ipm_options(max_iter=its, pcg=default_pcg_options(maxit=1))
    out = QP(spec).solve(opts, log=True)
    info = out["info"]
    assert info.result == 1 and info.iterations == its          # QP_IPM_MAX_ITER
    assert info.cg_maxiter_hits == its and info.total_cg_iters == its
    assert list(out["log"]["cg_iters"]) == [1] * its
    ref = O.solve(prob, O.IPMOptions(max_iter=its), direction=oracle_pcg_direction(1))
    assert ref.status == "max_iter"
    e = rel(out["x"].cpu().numpy(), ref.state.x)
    print(f"one-iteration PCG, {its} IPM steps: x differs from the oracle by {e:.2e}", flush=True)
    assert e <= 1e-10
    for k, le in enumerate(ref.log):
        assert out["log"]["mu"][k] == le["mu"]
        assert abs(out["log"]["rnorm"][k] - le["rnorm"]) <= 1e-10 * le["rnorm"]


@pytest.mark.gpu
def test_infeasible_rows_stop_at_the_ipm_cap():
    from paper_2308_00637_amd.qpk import QP, default_ipm_options
    spec = infeasible_case()
    out = QP(spec).solve(default_ipm_options(max_iter=8), log=True)
    info = out["info"]
    assert info.result == 1 and info.iterations == 8             # QP_IPM_MAX_ITER
    assert np.all(out["log"]["mu"] == 1.0) and np.all(out["log"]["rnorm"] >= 1.0)
    assert info.mu_final == 1.0
