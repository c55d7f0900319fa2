"""Shapes whose groups own more rows than they have lanes, so the passes that
keep each row's dot on a lane and run the epilogues in bursts flush several
times per group, not only after the group's last row:

* the blocked row pass (4 lanes per row) on 300,000 two-entry voxel rows of
  200 beamlets, about 4.6 rows per group;
* the single-chunk blocked column pass on 1,000,000 beamlets with two
  entries each, about 7.6 rows per group;
* the low-rank column pass (SVM form, no stored entries) and its general
  path (a low-rank H with dense rows of A) at 600,000 variables, past the
  524,288 at which a group of the capped grid owns more rows than lanes.

K v against the oracle's matrix-free product, and thirty CG iterations
against the oracle's PCG, step for step."""
import numpy as np
import pytest

import oracle as O
from oracle.pcg import pcg
from paper_2308_00637_amd import workloads as W
from tests.helpers import kkt_from_masked, kkt_to_masked, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "row_pass_300000x200": lambda: W.rt_qp(11, 300_000, 200, 0.01, 50, name="rt_300000x200"),
    "col_pass_2000x1000000": lambda: W.rt_qp(12, 2_000, 1_000_000, 0.001, 40,
                                             name="rt_2000x1000000"),
    "lowrank_svm_600000": lambda: W.svm_qp(13, 600_000, 4),
    "lowrank_rows_600000": lambda: W.qn_rt(14, 600_000, 4, 2),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    from paper_2308_00637_amd.qpk import QP
    spec = CASES[request.param]()
    prob = O.from_spec(spec)
    qp = QP(spec)
    print(f"case={request.param} n={prob.n} m={prob.m} me={prob.me} layout={qp.operator_layout()}",
          flush=True)
    return request.param, prob, qp


def test_kkt_matvec_against_oracle(case):
    name, prob, qp = case
    qp.init_state(1.0)
    st = O.initial_point(prob)
    S = O.index_sets(prob)
    v = np.random.default_rng(5).standard_normal(prob.n + prob.me + len(S.L) + len(S.U))
    y = kkt_from_masked(prob, qp.kkt_matvec(dev(kkt_to_masked(prob, v))).cpu().numpy())
    assert rel(y, O.kkt_matvec(prob, st, 1.0, v)) <= 1e-12


def test_thirty_cg_iterations_against_oracle(case):
    from paper_2308_00637_amd.qpk import default_pcg_options
    name, prob, qp = case
    qp.init_state(1.0)
    st = O.initial_point(prob)
    rhs, _ = qp.newton_rhs()
    ref_rhs, _ = O.newton_rhs_doubly(prob, st, 1.0)
    dg = O.jacobi_diagonal(prob, st, 1.0)
    x_ref, its, _, _ = pcg(lambda p: O.kkt_matvec(prob, st, 1.0, p), ref_rhs, dg, tol=1e-300, maxit=30)
    sol, info = qp.kkt_pcg_solve(rhs, default_pcg_options(maxit=30, tol=1e-300))
    assert its == 30 and info.iterations == 30
    err = rel(kkt_from_masked(prob, sol.cpu().numpy()), x_ref)
    print(f"{name}: 30 CG iterates differ by {err:.2e}", flush=True)
    assert err <= 1e-9
