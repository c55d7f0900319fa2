"""The fused single-read product of K v (qp_fused_layout): one pass over the
rows of P (and of A), the columns cut in two halves whose block pairs
exchange half dots, each entry used for the dot and the scatter.  Forced on
(QPK_FUSED=1) at shapes below its default size, against the oracle's
matrix-free functions and PCG; its fallback when a pair's bounded wait runs
out (QPK_FUSED_SPIN=1, a spin limit so small that the waits give up) is
checked to redo the work with the two-pass kernels.  The full-size
radiation-therapy QP runs it by default (test_gpu_fullsize)."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from oracle.pcg import pcg
from paper_2308_00637_amd import workloads as W
from tests.helpers import block_rel, from_masked, kkt_blocks, kkt_from_masked, kkt_to_masked

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ENV_KEYS = ("QPK_FUSED", "QPK_FUSED_SPIN", "QPK_FOLD_A")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def make_qp(spec, env, precision="fp64"):
    from paper_2308_00637_amd.qpk import QP
    old = {k: os.environ.get(k) for k in ENV_KEYS}
    try:
        for k in ENV_KEYS:
            os.environ.pop(k, None)
        os.environ.update({k: str(v) for k, v in env.items()})
        return QP(spec, precision=precision)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def with_equalities(spec, me, seed):
    """The radiation-therapy form plus `me` dense equality rows through a
    point of the feasible set (the penalty-barrier rows of eq. (3))."""
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((me, spec.n)) / np.sqrt(spec.n)
    x0 = rng.uniform(0.0, 0.02, spec.n)
    spec.C, spec.b = C, C @ x0
    return spec


CASES = {
    # max-dose rows folded into their twin rows of P; odd column count
    "rt_twins": (lambda: W.rt_qp(21, 12_001, 2_001, 0.01, 800, name="rt_12001x2001"), {}),
    # A kept as rows of its own after those of P
    "rt_rows_of_a": (lambda: W.rt_qp(22, 9_000, 1_500, 0.012, 600, name="rt_9000x1500"),
                     {"QPK_FOLD_A": 0}),
    # equality rows: their terms enter K v's x-part and p.q outside the pass
    "rt_equalities": (lambda: with_equalities(W.rt_qp(23, 8_000, 1_200, 0.01, 400,
                                                      name="rt_8000x1200"), 3, 23), {}),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    make, env = CASES[request.param]
    spec = make()
    prob = O.from_spec(spec)
    qp = make_qp(spec, {"QPK_FUSED": 1, **env})
    lay = qp.fused_layout()
    print(f"case={request.param} n={prob.n} m={prob.m} me={prob.me} fused={lay}", flush=True)
    assert lay["active"] and lay["ranges"] >= 1 and not lay["failed"]
    return request.param, spec, prob, qp


def test_fused_matvec_against_oracle(case):
    name, spec, prob, qp = case
    qp.init_state(1.0)
    st = O.initial_point(prob)
    rng = np.random.default_rng(31)
    N = sum(kkt_blocks(prob))
    for _ in range(2):
        v = rng.standard_normal(N)
        y = kkt_from_masked(prob, qp.kkt_matvec(dev(kkt_to_masked(prob, v))).cpu().numpy())
        assert block_rel(y, O.kkt_matvec(prob, st, 1.0, v), kkt_blocks(prob)) <= 1e-12
    assert not qp.fused_layout()["failed"]


def test_fused_thirty_cg_iterations_against_oracle(case):
    from paper_2308_00637_amd.qpk import default_pcg_options
    name, spec, prob, qp = case
    qp.init_state(1.0)
    st = O.initial_point(prob)
    rhs, _ = qp.newton_rhs()
    ref_rhs, _ = O.newton_rhs_doubly(prob, st, 1.0)
    dg = O.jacobi_diagonal(prob, st, 1.0)
    x_ref, its, _, _ = pcg(lambda p: O.kkt_matvec(prob, st, 1.0, p), ref_rhs, dg, tol=1e-300, maxit=30)
    sol, info = qp.kkt_pcg_solve(rhs, default_pcg_options(maxit=30, tol=1e-300))
    assert its == 30 and info.iterations == 30
    err = block_rel(kkt_from_masked(prob, sol.cpu().numpy()), x_ref, kkt_blocks(prob))
    print(f"{name}: 30 CG iterates differ by {err:.2e}", flush=True)
    assert err <= 1e-9
    assert not qp.fused_layout()["failed"]


def test_fused_ipm_solve_against_oracle(case):
    name, spec, prob, qp = case
    ref = O.solve(prob, direction=O.schur_direction)   # exact steps through the Schur complement
    out = qp.solve()
    info = out["info"]
    gst = from_masked(prob, out["x"].cpu().numpy(), out["lam"].cpu().numpy(), out["s"].cpu().numpy())
    kkt = O.stacked_norm(O.residuals(prob, gst, info.mu_final))
    err = abs(info.objective - ref.objective) / max(1.0, abs(ref.objective))
    print(f"{name}: ipm gpu={info.iterations} oracle={ref.iterations} cg={info.total_cg_iters} "
          f"obj err={err:.2e} kkt={kkt:.2e}", flush=True)
    assert info.result == 0 and err <= 1e-6 and kkt <= 1e-6
    assert not qp.fused_layout()["failed"]


def test_fused_adjoint_small_workload_against_stored_oracle_solution():
    """The 20,000 x 2,000 adjoint workload with the fused product forced on:
    the solve against the oracle's stored exact solution."""
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rt_small.json")) as fh:
        ref = json.load(fh)
    spec = W.rt_small(4)
    qp = make_qp(spec, {"QPK_FUSED": 1})
    assert qp.fused_layout()["active"]
    out = qp.solve()
    info = out["info"]
    err = abs(info.objective - ref["objective"]) / abs(ref["objective"])
    dx = float(np.max(np.abs(out["x"].cpu().numpy() - np.array(ref["x"]))))
    print(f"rt_small fused: ipm={info.iterations} cg={info.total_cg_iters} obj err={err:.2e} "
          f"max|dx|={dx:.2e}", flush=True)
    assert info.result == 0 and err <= 1e-6 and dx <= 1e-4


def test_fused_wait_timeout_falls_back_to_two_pass():
    """A spin limit of one poll makes the pairs' waits give up: the product is
    flagged invalid, the handle switches to the two-pass kernels for good and
    redoes the work, so every result is still right."""
    from paper_2308_00637_amd.qpk import default_pcg_options
    spec = W.rt_qp(24, 6_000, 1_000, 0.01, 300, name="rt_6000x1000")
    prob = O.from_spec(spec)
    qp = make_qp(spec, {"QPK_FUSED": 1, "QPK_FUSED_SPIN": 1})
    assert qp.fused_layout()["active"]
    qp.init_state(1.0)
    st = O.initial_point(prob)
    v = np.random.default_rng(2).standard_normal(sum(kkt_blocks(prob)))
    y = kkt_from_masked(prob, qp.kkt_matvec(dev(kkt_to_masked(prob, v))).cpu().numpy())
    lay = qp.fused_layout()
    print(f"after one product with a one-poll wait limit: {lay}", flush=True)
    assert block_rel(y, O.kkt_matvec(prob, st, 1.0, v), kkt_blocks(prob)) <= 1e-12
    if lay["failed"]:
        assert not lay["active"]
    # a PCG solve and a whole IPM solve on the same handle stay right either way
    rhs, _ = qp.newton_rhs()
    ref_rhs, _ = O.newton_rhs_doubly(prob, st, 1.0)
    sol, info = qp.kkt_pcg_solve(rhs, default_pcg_options(tol=1e-10, maxit=5000))
    solc = kkt_from_masked(prob, sol.cpu().numpy())
    true_rel = np.linalg.norm(ref_rhs - O.kkt_matvec(prob, st, 1.0, solc)) / np.linalg.norm(ref_rhs)
    assert info.converged == 1 and true_rel <= 1.5e-10
    ref = O.solve(prob, direction=O.schur_direction)
    out = qp.solve()
    assert out["info"].result == 0
    assert abs(out["info"].objective - ref.objective) <= 1e-6 * max(1.0, abs(ref.objective))


@pytest.mark.parametrize("prec", ["fp32x64", "bf16"])
def test_fused_reduced_precision_pcg(prec):
    """Reduced-precision operator values in the fused pass: the PCG solve is
    accepted on the float64 residual, as with the two-pass kernels."""
    from paper_2308_00637_amd.qpk import default_pcg_options
    spec = W.rt_qp(25, 8_000, 1_500, 0.01, 500, name="rt_8000x1500")
    prob = O.from_spec(spec)
    qp = make_qp(spec, {"QPK_FUSED": 1}, precision=prec)
    assert qp.fused_layout()["active"]
    qp.init_state(1.0)
    st = O.initial_point(prob)
    rhs, _ = qp.newton_rhs()
    sol, info = qp.kkt_pcg_solve(rhs, default_pcg_options(tol=1e-9, maxit=20000))
    ref_rhs, _ = O.newton_rhs_doubly(prob, st, 1.0)
    solc = kkt_from_masked(prob, sol.cpu().numpy())
    true_rel = np.linalg.norm(ref_rhs - O.kkt_matvec(prob, st, 1.0, solc)) / np.linalg.norm(ref_rhs)
    print(f"{prec}: iters={info.iterations} relres={info.rel_residual:.2e} true={true_rel:.2e} "
          f"escalated={info.escalated}", flush=True)
    assert info.converged == 1 and true_rel <= 1.5e-9
