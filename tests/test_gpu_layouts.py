"""The blocked operator layouts and their kernel variants, on a radiation-
therapy-shaped QP wide enough that both sides of K v need several LDS chunks
(24,001 beamlets > 20,224 columns per row-side chunk; 42,001 voxel and
max-dose rows > 10,112 columns per column-side chunk; both last chunks have
odd width), so every PCG product runs the per-chunk partial kernels and both
epilogues.  Against the oracle's
matrix-free functions, and against each other: the staging variants and the
two row directions change no arithmetic, so their products agree bitwise.  Every max-dose row of A repeats a row of P,
so by default both passes hold P alone (the A-row epilogues run on the twin
P rows' dots); QPK_FOLD_A=0 keeps A in both passes, and the two must agree to
rounding."""
import dataclasses
import os

import numpy as np
import pytest

import oracle as O
from paper_2308_00637_amd import workloads as W
from tests.helpers import from_masked, kkt_from_masked, kkt_to_masked, rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def wide():
    # odd sizes: the last chunk of either side has an odd width
    spec = W.rt_qp(5, 40_001, 24_001, 0.002, 2_000, name="rt_wide_40001x24001")
    return spec, O.from_spec(spec)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def make_qp(spec, env):
    from paper_2308_00637_amd.qpk import QP
    keys = ("QPK_KV_R", "QPK_KV_X", "QPK_ALTERNATE", "QPK_FOLD_A", "QPK_CHUNK_COLS_R",
            "QPK_CHUNK_COLS_X")
    old = {k: os.environ.get(k) for k in keys}
    try:
        for k in keys:
            os.environ.pop(k, None)
        os.environ.update({k: str(v) for k, v in env.items()})
        return QP(spec)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_wide_layout_is_multi_chunk_on_both_sides(wide):
    spec, _ = wide
    lay = make_qp(spec, {}).operator_layout()
    print(lay, flush=True)
    assert lay["row"]["chunks"] == 2 and lay["col"]["chunks"] >= 4


def test_wide_matvec_and_pcg_against_oracle(wide):
    spec, prob = wide
    qp = make_qp(spec, {})
    qp.init_state(1.0)
    st = O.initial_point(prob)
    rhs, dg = qp.newton_rhs()
    ref_rhs, _ = O.newton_rhs_doubly(prob, st, 1.0)
    assert rel(kkt_from_masked(prob, rhs.cpu().numpy()), ref_rhs) <= 1e-12
    assert rel(kkt_from_masked(prob, dg.cpu().numpy()), O.jacobi_diagonal(prob, st, 1.0)) <= 1e-12
    v = np.random.default_rng(1).standard_normal(ref_rhs.size)
    y = qp.kkt_matvec(dev(kkt_to_masked(prob, v)))
    assert rel(kkt_from_masked(prob, y.cpu().numpy()), O.kkt_matvec(prob, st, 1.0, v)) <= 1e-12
    sol, info = qp.kkt_pcg_solve(rhs)
    assert info.converged == 1
    solc = kkt_from_masked(prob, sol.cpu().numpy())
    true_rel = np.linalg.norm(ref_rhs - O.kkt_matvec(prob, st, 1.0, solc)) / np.linalg.norm(ref_rhs)
    print(f"pcg iters={info.iterations} true relres={true_rel:.3e}", flush=True)
    assert true_rel <= 1.5e-7


@pytest.mark.parametrize("env", [{"QPK_KV_R": 0}, {"QPK_KV_X": 0}, {"QPK_ALTERNATE": 0}])
def test_variants_and_directions_agree_bitwise(wide, env):
    spec, prob = wide
    base = make_qp(spec, {})
    other = make_qp(spec, env)
    v = dev(kkt_to_masked(prob, np.random.default_rng(2).standard_normal(
        prob.n + prob.me + len(O.index_sets(prob).L) + len(O.index_sets(prob).U))))
    for qp in (base, other):
        qp.init_state(1.0)
        qp.newton_rhs()
    # two products in a row: the default alternates the row direction between them
    y0, y1 = base.kkt_matvec(v), base.kkt_matvec(v)
    z0, z1 = other.kkt_matvec(v), other.kkt_matvec(v)
    assert torch.equal(y0, y1)
    assert torch.equal(y0, z0) and torch.equal(y0, z1)


def test_wide_ipm_solve_kkt_by_oracle_function(wide):
    spec, prob = wide
    qp = make_qp(spec, {})
    out = qp.solve()
    info = out["info"]
    print(f"ipm={info.iterations} cg={info.total_cg_iters} time={info.time_ms / 1e3:.2f}s "
          f"rnorm={info.rnorm:.3e}", flush=True)
    assert info.result == 0 and info.mu_final < 1e-6
    gst = from_masked(prob, out["x"].cpu().numpy(), out["lam"].cpu().numpy(), out["s"].cpu().numpy())
    kkt = O.stacked_norm(O.residuals(prob, gst, info.mu_final))
    assert kkt <= 1e-6 and kkt == pytest.approx(info.rnorm, rel=1e-9)
    assert info.objective == pytest.approx(O.objective(prob, gst.x), rel=1e-12)


def test_twin_rows_fold_against_unfolded_and_oracle(wide):
    spec, prob = wide
    folded, plain = make_qp(spec, {}), make_qp(spec, {"QPK_FOLD_A": 0})
    bf, bp = folded.operator_bytes(), plain.operator_bytes()
    print(f"folded row/col bytes {bf['row_bytes']}/{bf['col_bytes']}, "
          f"unfolded {bp['row_bytes']}/{bp['col_bytes']}", flush=True)
    # A (2,000 rows of ~48 entries) is streamed by neither folded pass
    assert bf["row_bytes"] < bp["row_bytes"] and bf["col_bytes"] < bp["col_bytes"]
    st = O.initial_point(prob)
    S = O.index_sets(prob)
    v = np.random.default_rng(3).standard_normal(prob.n + prob.me + len(S.L) + len(S.U))
    ref = O.kkt_matvec(prob, st, 1.0, v)
    ys = []
    for qp in (folded, plain):
        qp.init_state(1.0)
        qp.newton_rhs()
        y = kkt_from_masked(prob, qp.kkt_matvec(dev(kkt_to_masked(prob, v))).cpu().numpy())
        assert rel(y, ref) <= 1e-12
        ys.append(y)
    assert rel(ys[0], ys[1]) <= 1e-14
    its = []
    for qp in (folded, plain):
        rhs, _ = qp.newton_rhs()
        sol, info = qp.kkt_pcg_solve(rhs)
        assert info.converged == 1
        its.append(info.iterations)
    print(f"pcg iterations folded {its[0]}, unfolded {its[1]}", flush=True)
    assert abs(its[0] - its[1]) <= max(2, its[1] // 50)


def test_no_fold_when_one_a_row_differs(wide):
    spec, prob = wide
    A = spec.A.copy()
    A.data = A.data.copy()
    A.data[A.indptr[7]] *= 1.0 + 2.0 ** -40   # row 7 no longer repeats its P row
    spec2 = dataclasses.replace(spec, A=A, name="rt_wide_one_row_off")
    prob2 = O.from_spec(spec2)
    qp, plain = make_qp(spec2, {}), make_qp(spec2, {"QPK_FOLD_A": 0})
    assert qp.operator_bytes() == plain.operator_bytes()
    st = O.initial_point(prob2)
    S = O.index_sets(prob2)
    v = np.random.default_rng(4).standard_normal(prob2.n + prob2.me + len(S.L) + len(S.U))
    qp.init_state(1.0)
    qp.newton_rhs()
    y = kkt_from_masked(prob2, qp.kkt_matvec(dev(kkt_to_masked(prob2, v))).cpu().numpy())
    assert rel(y, O.kkt_matvec(prob2, st, 1.0, v)) <= 1e-12


def _rt_with_rows(P, rows, seed):
    """A radiation-therapy QP on P whose max-dose rows are the given rows of P."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    n_vox, n = P.shape
    A = sp.csr_matrix(P[rows])
    return W.QPSpec(n=n, c=np.zeros(n), h_kind="ptwp", P=P, w=np.where(rng.random(n_vox) < 0.1, 10.0, 1.0),
                    d=rng.uniform(0.0, 1.0, n_vox), A=A, lA=np.full(len(rows), -np.inf),
                    uA=np.full(len(rows), 0.8), lx=np.zeros(n), ux=np.full(n, np.inf))


@pytest.mark.parametrize("kind", ["repeated_a_row", "repeated_p_row"])
def test_twin_rows_with_repeats(kind):
    """Two equal rows of A and one such row of P: no fold (each A row needs
    a twin of its own); two equal rows of P repeated by two rows of A: fold,
    one twin each.  Either way K v matches the oracle."""
    import scipy.sparse as sp
    base = W.rt_qp(21, 3_000, 400, 0.02, 1, name="rt_repeats")
    P = sp.csr_matrix(base.P)
    if kind == "repeated_a_row":
        rows, fold = [5, 9, 9, 40], False
    else:
        P = sp.vstack([P, P[[17]]]).tocsr()   # row 3,000 repeats row 17
        rows, fold = [17, 3_000, 40], True
    spec = _rt_with_rows(P, rows, 22)
    prob = O.from_spec(spec)
    qp, plain = make_qp(spec, {}), make_qp(spec, {"QPK_FOLD_A": 0})
    bf, bp = qp.operator_bytes(), plain.operator_bytes()
    assert (bf["col_bytes"] < bp["col_bytes"]) == fold
    st = O.initial_point(prob)
    S = O.index_sets(prob)
    v = np.random.default_rng(6).standard_normal(prob.n + prob.me + len(S.L) + len(S.U))
    qp.init_state(1.0)
    qp.newton_rhs()
    y = kkt_from_masked(prob, qp.kkt_matvec(dev(kkt_to_masked(prob, v))).cpu().numpy())
    assert rel(y, O.kkt_matvec(prob, st, 1.0, v)) <= 1e-12


NARROW = {
    # single-chunk column side (15 dense rows of A), narrowest chunks: more
    # than kGridMax work items unless the builder caps them
    "lowrank_rows_1024": lambda: W.qn_rt(15, 30_000, 4, 15),
    # several chunks on both sides at the narrowest width
    "rt_1024": lambda: W.rt_qp(16, 6_001, 3_001, 0.01, 600, name="rt_6001x3001"),
}


@pytest.mark.parametrize("name", list(NARROW))
def test_narrowest_chunks_stay_within_partial_slots(name):
    """QPK_CHUNK_COLS_R/_X = 1024 (the narrowest chunk width): the work items
    of every pass fit the 2048 partial-sum slots, and K v and thirty CG
    iterations still match the oracle."""
    from oracle.pcg import pcg
    from paper_2308_00637_amd.qpk import default_pcg_options
    spec = NARROW[name]()
    prob = O.from_spec(spec)
    qp = make_qp(spec, {"QPK_CHUNK_COLS_R": 1024, "QPK_CHUNK_COLS_X": 1024})
    lay = qp.operator_layout()
    print(f"case={name} layout={lay}", flush=True)
    assert all(lay[side]["work_items"] <= 2048 for side in ("row", "col"))
    assert any(lay[side]["chunk_cols"] == 1024 for side in ("row", "col"))
    qp.init_state(1.0)
    st = O.initial_point(prob)
    v = np.random.default_rng(3).standard_normal(prob.n + prob.me + len(O.index_sets(prob).L)
                                                 + len(O.index_sets(prob).U))
    y = kkt_from_masked(prob, qp.kkt_matvec(dev(kkt_to_masked(prob, v))).cpu().numpy())
    assert rel(y, O.kkt_matvec(prob, st, 1.0, v)) <= 1e-12
    rhs, _ = qp.newton_rhs()
    ref_rhs, _ = O.newton_rhs_doubly(prob, st, 1.0)
    dg = O.jacobi_diagonal(prob, st, 1.0)
    x_ref, its, _, _ = pcg(lambda p: O.kkt_matvec(prob, st, 1.0, p), ref_rhs, dg, tol=1e-300, maxit=30)
    sol, info = qp.kkt_pcg_solve(rhs, default_pcg_options(maxit=30, tol=1e-300))
    assert its == 30 and info.iterations == 30
    err = rel(kkt_from_masked(prob, sol.cpu().numpy()), x_ref)
    print(f"{name}: 30 CG iterates differ by {err:.2e}", flush=True)
    assert err <= 1e-9
