"""SVM-dual workload (H = Z Z^T applied as two tall-skinny passes, one
equality row y^T alpha = 0, box 0 <= alpha <= 1) against the exact Woodbury
oracle.  alpha* is not unique (Z Z^T has rank 128), so the checks compare what
is: the objective, the primal weight w = Z^T alpha, and the KKT residual by the
oracle's own function."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2308_00637_amd import workloads as W
from tests.helpers import from_masked, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "svm_full.json")


def check(spec, out, obj_ref, w_ref):
    prob = O.from_spec(spec)
    info = out["info"]
    assert info.result == 0
    alpha = out["x"].cpu().numpy()
    st = from_masked(prob, alpha, out["lam"].cpu().numpy(), out["s"].cpu().numpy())
    kkt = O.stacked_norm(O.residuals(prob, st, info.mu_final))
    werr = rel(spec.U.T @ alpha, w_ref)
    print(f"{spec.name}: ipm={info.iterations} cg={info.total_cg_iters} time={info.time_ms / 1e3:.2f}s "
          f"obj={info.objective:.12g} ref={obj_ref:.12g} kkt={kkt:.2e} w_err={werr:.2e}", flush=True)
    assert abs(info.objective - obj_ref) <= 1e-6 * max(1.0, abs(obj_ref))
    assert kkt <= 1e-6
    assert werr <= 1e-4
    assert alpha.min() >= -1e-9 and alpha.max() <= 1 + 1e-9
    assert abs(spec.extra["y"] @ alpha) <= 1e-5


def test_svm_downscaled_against_woodbury_oracle():
    from paper_2308_00637_amd.qpk import QP
    spec = W.svm_qp(2, 20000, 128, name="svm_20000x128")
    prob = O.from_spec(spec)
    d = lambda pr, st, mu, res: O.woodbury_direction(pr, st, mu, res, h0=spec.h0, U=spec.U, wd=spec.wd)
    ref = O.solve(prob, direction=d)
    out = QP(spec).solve()
    check(spec, out, ref.objective, spec.U.T @ ref.state.x)


@pytest.mark.slow
def test_svm_full_against_stored_oracle_result():
    from paper_2308_00637_amd.qpk import QP
    g = json.load(open(GOLDEN))
    spec = W.svm_full()
    out = QP(spec).solve()
    check(spec, out, g["objective"], np.array(g["w_svm"]))


def test_svm_rbf_at_a1a_shape_against_dense_oracle():
    """Dense precomputed RBF-kernel Hessian, 1,605 samples (the a1a shape of
    Table 1), against the dense oracle's full solve."""
    from paper_2308_00637_amd.qpk import QP
    spec = W.svm_rbf(7)
    prob = O.from_spec(spec)
    ref = O.solve(prob)
    out = QP(spec).solve()
    info = out["info"]
    alpha = out["x"].cpu().numpy()
    st = from_masked(prob, alpha, out["lam"].cpu().numpy(), out["s"].cpu().numpy())
    kkt = O.stacked_norm(O.residuals(prob, st, info.mu_final))
    print(f"svm_rbf: ipm={info.iterations} (oracle {ref.iterations}) cg={info.total_cg_iters} "
          f"time={info.time_ms / 1e3:.2f}s obj={info.objective:.12g} ref={ref.objective:.12g} "
          f"kkt={kkt:.2e}", flush=True)
    assert info.result == 0 and ref.status == "converged"
    assert abs(info.objective - ref.objective) <= 1e-6 * max(1.0, abs(ref.objective))
    assert kkt <= 1e-6
    assert rel(alpha, ref.state.x) <= 1e-3
    assert alpha.min() >= -1e-9 and alpha.max() <= 1 + 1e-9
