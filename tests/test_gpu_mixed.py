"""Reduced-precision PCG matvec (operator values in float32 or bfloat16,
float32 accumulation) with float64 reductions, float64 residual replacement
and a float64 acceptance test: parity with the float64 oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2308_00637_amd import workloads as W
from tests.helpers import from_masked, kkt_from_masked, random_state, rel, to_masked

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    "rt_ptwp": lambda: W.rt_qp(5, 700, 61, 0.08, 23, maxdose=0.6),
    "general_csr_lowrank": lambda: W.random_bounded_qp(2, 53, 41, 1, 9, a_sparse=True, h_kind="lowrank"),
    "svm_lowrank_eq": lambda: W.svm_qp(6, 333, 7),
}


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp32x64", "bf16x64"])
@pytest.mark.parametrize("case", list(CASES))
def test_mixed_pcg_meets_tolerance_on_float64_residual(case, prec):
    from paper_2308_00637_amd.qpk import QP, default_pcg_options
    spec = CASES[case]()
    prob = O.from_spec(spec)
    st = random_state(prob, np.random.default_rng(3), 0.5)
    qp = QP(spec, precision=prec)
    x, lam, s = to_masked(prob, st)
    qp.set_state(dev(x), dev(lam), dev(s), 0.05)
    rhs, _ = qp.newton_rhs()
    sol, info = qp.kkt_pcg_solve(rhs, default_pcg_options(tol=1e-9, maxit=20000))
    print(f"{case} {prec}: iters={info.iterations} relres={info.rel_residual:.2e} "
          f"escalated={info.escalated}", flush=True)
    assert info.converged == 1 and info.rel_residual <= 1e-9
    ref_rhs, res = O.newton_rhs_doubly(prob, st, 0.05)
    Q, B, D, r1, r2, _ = O.reduced_system(prob, st, res, 0.05)
    K, _ = O.doubly_augmented(Q, B, D, r1, r2)
    assert rel(kkt_from_masked(prob, sol.cpu().numpy()), np.linalg.solve(K, ref_rhs)) <= 1e-6


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp32x64", "bf16x64"])
@pytest.mark.parametrize("case", list(CASES))
def test_mixed_ipm_matches_oracle(case, prec):
    from paper_2308_00637_amd.qpk import QP
    spec = CASES[case]()
    prob = O.from_spec(spec)
    ref = O.solve(prob)
    out = QP(spec, precision=prec).solve()
    info = out["info"]
    gst = from_masked(prob, out["x"].cpu().numpy(), out["lam"].cpu().numpy(), out["s"].cpu().numpy())
    kkt = O.stacked_norm(O.residuals(prob, gst, info.mu_final))
    err = abs(info.objective - ref.objective) / max(1.0, abs(ref.objective))
    print(f"{case} {prec}: ipm={info.iterations} cg={info.total_cg_iters} obj_err={err:.2e} kkt={kkt:.2e} "
          f"escalations={info.cg_escalations}", flush=True)
    assert info.result == 0
    assert kkt <= 1e-6
    assert err <= 1e-6
