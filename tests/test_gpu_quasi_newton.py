"""Quasi-Newton Hessian at the proton-liver shape of Table 1: 90,657
variables, H = diag(h0) + U diag(w) U^T with k = 20 and mixed-sign w, 15
two-sided general rows, x >= 0.  The dense oracle cannot run at this size, so
the checks use the oracle's matrix-free functions (residuals, right-hand side,
Jacobi diagonal, K v) and properties that hold at any size; the mixed-sign
form is checked step by step against the dense oracle at n = 300 in
test_gpu_steps."""
import numpy as np
import pytest

import oracle as O
from paper_2308_00637_amd import workloads as W
from tests.helpers import from_masked, kkt_from_masked, kkt_to_masked, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def qn():
    from paper_2308_00637_amd.qpk import QP
    spec = W.qn_rt()
    assert (spec.wd < 0).any() and (spec.wd > 0).any()
    return spec, O.from_spec(spec), QP(spec)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_qn_steps_at_start_point(qn):
    spec, prob, qp = qn
    qp.init_state(1.0)
    st = O.initial_point(prob)
    rhs, dg = qp.newton_rhs()
    ref_rhs, _ = O.newton_rhs_doubly(prob, st, 1.0)
    assert rel(kkt_from_masked(prob, rhs.cpu().numpy()), ref_rhs) <= 1e-12
    assert rel(kkt_from_masked(prob, dg.cpu().numpy()), O.jacobi_diagonal(prob, st, 1.0)) <= 1e-12
    v = np.random.default_rng(3).standard_normal(ref_rhs.size)
    y = qp.kkt_matvec(dev(kkt_to_masked(prob, v)))
    assert rel(kkt_from_masked(prob, y.cpu().numpy()), O.kkt_matvec(prob, st, 1.0, v)) <= 1e-12
    sol, info = qp.kkt_pcg_solve(rhs)
    assert info.converged == 1
    solc = kkt_from_masked(prob, sol.cpu().numpy())
    true_rel = np.linalg.norm(ref_rhs - O.kkt_matvec(prob, st, 1.0, solc)) / np.linalg.norm(ref_rhs)
    assert true_rel <= 1.5e-7, true_rel


def test_qn_ipm_solve_kkt_by_oracle_function(qn):
    spec, prob, qp = qn
    out = qp.solve()
    info = out["info"]
    print(f"ipm={info.iterations} cg={info.total_cg_iters} caps={info.cg_maxiter_hits} "
          f"time={info.time_ms / 1e3:.2f}s rnorm={info.rnorm:.3e}", flush=True)
    assert info.result == 0 and info.mu_final < 1e-6
    gst = from_masked(prob, out["x"].cpu().numpy(), out["lam"].cpu().numpy(), out["s"].cpu().numpy())
    kkt = O.stacked_norm(O.residuals(prob, gst, info.mu_final))
    assert kkt <= 1e-6 and kkt == pytest.approx(info.rnorm, rel=1e-9)
    assert info.objective == pytest.approx(O.objective(prob, gst.x), rel=1e-12)
    assert gst.x.min() >= -1e-9
    ax = spec.A @ gst.x
    assert (ax >= spec.lA - 1e-6).all() and (ax <= spec.uA + 1e-6).all()
