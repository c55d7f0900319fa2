"""PCG chunks replayed from a HIP graph (qp_graph_stats): a handle built with
QPK_GRAPH=0 launches every kernel itself, the default one captures a chunk
of iterations once per Newton system and replays it.  The kernels and their
arguments are the same, so on the deterministic layouts the solves agree
bit for bit, on the fused pass (whose LDS atomics add in a run-dependent
order) to rounding; every replay is checked, with the program's own eager
kernels and synchronisations between replays."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2308_00637_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = {
    # equality rows: the product takes mu by value, so each new mu recaptures
    "general_dense_eq": (lambda: W.random_bounded_qp(1, 37, 29, 2, 11), {}, True),
    "quasi_newton": (lambda: W.qn_rt(6, 300, 12, 15), {}, True),
    "rt_small_two_pass": (W.rt_small, {"QPK_FUSED": 0}, True),
    "rt_fused": (lambda: W.rt_qp(21, 12_001, 2_001, 0.01, 800, name="rt_12001x2001"),
                 {"QPK_FUSED": 1}, False),
}
KEYS = ("QPK_GRAPH", "QPK_FUSED")


def make_qp(spec, env):
    from paper_2308_00637_amd.qpk import QP
    old = {k: os.environ.get(k) for k in KEYS}
    try:
        for k in KEYS:
            os.environ.pop(k, None)
        os.environ.update({k: str(v) for k, v in env.items()})
        return QP(spec)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("case", list(CASES))
def test_graph_replays_match_kernel_by_kernel_launches(case):
    from paper_2308_00637_amd.qpk import default_pcg_options
    make, env, exact = CASES[case]
    spec = make()
    g = make_qp(spec, {**env})
    e = make_qp(spec, {**env, "QPK_GRAPH": 0})
    # repeated PCG solves on one state: every replay against the eager solve
    for q in (g, e):
        q.init_state(1.0)
    rhs_g, _ = g.newton_rhs()
    rhs_e, _ = e.newton_rhs()
    for rep in range(3):
        sg, ig = g.kkt_pcg_solve(rhs_g, default_pcg_options(tol=1e-9))
        se, ie = e.kkt_pcg_solve(rhs_e, default_pcg_options(tol=1e-9))
        torch.cuda.synchronize()
        d = float(torch.max(torch.abs(sg - se))) / max(1e-300, float(torch.max(torch.abs(se))))
        assert ig.converged == ie.converged == 1
        if exact:
            assert ig.iterations == ie.iterations and d == 0.0, (rep, d)
        else:   # run-dependent rounding can move the stop by one iteration
            assert abs(ig.iterations - ie.iterations) <= 1 and d <= 1e-6, (rep, d)
    # whole solves: eager residual, right-hand side and recovery kernels and a
    # host read-back between the replays of every Newton system
    og, oe = g.solve(), e.solve()
    cg, rg = g.graph_stats()
    ce, re_ = e.graph_stats()
    a, b = og["info"], oe["info"]
    dx = float(torch.max(torch.abs(og["x"] - oe["x"])))
    print(f"{case}: graph {a.time_ms:.1f} ms ({cg} captures, {rg} replays) vs eager {b.time_ms:.1f} ms; "
          f"ipm {a.iterations}/{b.iterations} cg {a.total_cg_iters}/{b.total_cg_iters} max|dx| {dx:.1e}",
          flush=True)
    assert cg >= 2 and rg > cg and ce == 0 and re_ == 0
    assert a.result == 0 and b.result == 0
    if exact:
        assert a.iterations == b.iterations and a.total_cg_iters == b.total_cg_iters
        assert torch.equal(og["x"], oe["x"]) and a.objective == b.objective
    else:
        # the fused pass's run-dependent rounding can part the two IPM paths
        # late (one Newton step more or less): the same optimum to the
        # accuracy the barrier leaves (x to about sqrt(mu), mu ~ 1e-7)
        assert abs(a.iterations - b.iterations) <= 1 and dx <= 1e-4
        assert a.objective == pytest.approx(b.objective, rel=1e-7)
    ref = O.solve(O.from_spec(spec)) if spec.n <= 400 else None
    if ref is not None:
        assert a.objective == pytest.approx(ref.objective, rel=1e-6, abs=1e-9)
